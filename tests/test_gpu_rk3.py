"""The device time-step on a brick: ghost fill, full and face ghosts only
(bitwise, against the brick oracle), and the three SSP-RK3 stages (per
stage, against the oracle's composition of its own hydro stage, on the
interiors and face ghosts the time-step fills: for 8^3 sub-grids the stage
kernels write the face ghosts from their own stores, other edges run the
fill kernel), the graph form (bitwise the launches), and Sod's shock tube
converging on the GPU."""
import numpy as np
import pytest

from oracle import brick as ob
from paper_2210_06438_amd import hydroagg, workloads
from tests.gpu_util import normwise_each
from tests.ref import euler, riemann

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _nan_ghosts(rng, nb, n, nf):
    M = n + 6
    U = np.full((nb[0] * nb[1] * nb[2], nf, M, M, M), np.nan)
    U[:, :, 3:3 + n, 3:3 + n, 3:3 + n] = rng.uniform(0.5, 1.5, size=(len(U), nf, n, n, n))
    return U


@pytest.mark.parametrize("n,nf,nb,bc", [
    (8, 6, (2, 2, 2), (0, 0, 0)),
    (8, 11, (3, 2, 1), (1, 0, 0)),
    (12, 11, (1, 2, 3), (1, 1, 1)),
    (16, 6, (2, 1, 2), (0, 1, 0)),
    (8, 11, (1, 1, 1), (0, 0, 1)),
])
def test_ghost_fill_is_bitwise_the_oracle(dev, n, nf, nb, bc):
    rng = np.random.default_rng(n + nf + sum(nb))
    U = _nan_ghosts(rng, nb, n, nf)
    u = torch.from_numpy(U).to(dev)
    print(f"fill: n={n} F={nf} nb={nb} bc={bc}", flush=True)
    hydroagg.ghost_fill(hydroagg.brick(n, nf, nb, bc), u)
    torch.cuda.synchronize()
    assert np.array_equal(u.cpu().numpy(), ob.ghost_fill(U, nb, bc))


def _face_mask(n):
    """Cells of the stored block that are interior or face ghosts (at most one
    coordinate outside the interior)."""
    M = n + 6
    c = np.arange(M)
    out = (c < 3) | (c >= 3 + n)
    Z, Y, X = np.meshgrid(out, out, out, indexing="ij")
    return (Z.astype(int) + Y + X) <= 1


@pytest.mark.parametrize("n,nf,nb,bc", [
    (8, 11, (2, 2, 2), (0, 0, 0)),
    (12, 6, (3, 1, 2), (1, 0, 1)),
    (16, 11, (1, 2, 1), (0, 1, 1)),
])
def test_face_ghost_fill_is_bitwise_the_oracle_on_face_ghosts(dev, n, nf, nb, bc):
    """Face ghosts equal the oracle's fill bitwise; edge and corner ghosts
    keep what they held (NaN here)."""
    rng = np.random.default_rng(7 * n + nf + sum(nb))
    U = _nan_ghosts(rng, nb, n, nf)
    u = torch.from_numpy(U).to(dev)
    print(f"face fill: n={n} F={nf} nb={nb} bc={bc}", flush=True)
    hydroagg.ghost_fill_faces(hydroagg.brick(n, nf, nb, bc), u)
    torch.cuda.synchronize()
    got = u.cpu().numpy()
    want = ob.ghost_fill(U, nb, bc)
    m = _face_mask(n)
    assert np.array_equal(got[..., m], want[..., m])
    assert np.all(np.isnan(got[..., ~m]))


def _sod_brick(nsub, n=8):
    """Sod's shock tube on a strip of nsub sub-grids (outflow in x, periodic
    in y and z), ghosts filled by the oracle."""
    cells = n * nsub
    x = (np.arange(cells) + 0.5) / cells
    W = np.zeros((6, n, n, cells))
    left = x < 0.5
    W[0] = np.where(left, 1.0, 0.125)
    W[4] = np.where(left, 1.0, 0.1)
    W[5] = 1.0
    G = euler.cons(W)
    M = n + 6
    U = np.full((nsub, 6, M, M, M), np.nan)
    for s in range(nsub):
        U[s, :, 3:3 + n, 3:3 + n, 3:3 + n] = G[..., s * n:(s + 1) * n]
    return ob.ghost_fill(U, (nsub, 1, 1), (1, 0, 0)), x


CASES = {
    "periodic_brick": lambda: (workloads.brick(seed=1), (2, 2, 2), (0, 0, 0), 1 / 64, 0),
    "sod_strip": lambda: (_sod_brick(8)[0], (8, 1, 1), (1, 0, 0), 1 / 64, 0),
    "random_11_fields_level_1": lambda: (
        ob.ghost_fill(workloads.random_smooth(6, n=8, nfields=11, seed=31), (3, 1, 2), (1, 0, 1)),
        (3, 1, 2), (1, 0, 1), 0.1, 1),
    # one sub-grid across the outflow axes: both edges of x and z are the
    # domain's, so every face ghost there comes from the sub-grid itself
    "outflow_single_layers": lambda: (
        ob.ghost_fill(workloads.random_smooth(2, n=8, nfields=6, seed=33), (1, 2, 1), (1, 0, 1)),
        (1, 2, 1), (1, 0, 1), 0.1, 0),
    # 12^3 sub-grids: the steps and the stage combinations as separate kernels
    "random_12_cubed": lambda: (
        ob.ghost_fill(workloads.random_smooth(4, n=12, nfields=11, seed=32), (2, 2, 1), (0, 1, 0)),
        (2, 2, 1), (0, 1, 0), 0.1, 0),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_rk3_stages_match_the_oracle(dev, oracle_mod, case):
    U0, nb, bc, dx, level = CASES[case]()
    count, nf, M = U0.shape[0], U0.shape[1], U0.shape[2]
    n = M - 6
    levels = [level] * count
    _, a = oracle_mod.step(U0, 0.0, dx, levels=levels)
    dt = 0.4 * dx * 2.0 ** (-level) / a.max()
    ref = ob.rk3_stages(lambda V: oracle_mod.step(V, dt, dx, levels=levels)[0], U0, nb, bc)
    u = torch.from_numpy(U0).to(dev)
    w = torch.full_like(u, float("nan"))
    s = torch.full_like(u, float("nan"))
    amax = torch.zeros(count, dtype=torch.float64, device=dev)
    b = hydroagg.brick(n, nf, nb, bc, level)
    rk = hydroagg.RK3(b, u, w, s)
    try:
        for k in (1, 2, 3):
            print(f"rk3 {case}: stage {k}", flush=True)
            rk.stage(k, dt, dx, amax if k == 1 else None)
            torch.cuda.synchronize()
            out = {1: w, 2: s, 3: u}[k]                   # U1 in w, U2 in s, U3 in u
            got = out.cpu().numpy()
            # the face ghosts the stage left are bitwise what the fill kernel
            # copies from the interiors it formed
            refill = out.clone()
            hydroagg.ghost_fill_faces(b, refill)
            torch.cuda.synchronize()
            assert np.array_equal(refill.cpu().numpy(), got, equal_nan=True), k
            # the stage fills face ghosts only (the only ghosts the next
            # stage reads): compare interiors and face ghosts; the work
            # buffers' edge and corner ghosts stay as they were (NaN)
            m = _face_mask(n)
            err = normwise_each(got[..., m], ref[k - 1][..., m])
            if k < 3:
                assert np.all(np.isnan(got[..., ~m]))
            print(f"  worst per-sub-grid normwise {err.max():.2e}", flush=True)
            assert np.all(err <= TOL), (k, err.max())
            if k == 1:
                assert np.max(np.abs(amax.cpu().numpy() - a) / a) <= 1e-13
    finally:
        rk.close()


def test_rk3_graph_is_bitwise_the_launches(dev):
    U0 = workloads.brick(seed=9)
    nb, bc, dx = (2, 2, 2), (0, 0, 0), 1 / 64
    dt = 2e-3
    u = torch.from_numpy(U0).to(dev)
    w, s = torch.empty_like(u), torch.empty_like(u)
    amax = torch.zeros(8, dtype=torch.float64, device=dev)
    rk = hydroagg.RK3(hydroagg.brick(8, 6, nb, bc), u, w, s)
    try:
        for _ in range(2):
            rk.step(dt, dx, amax)
        torch.cuda.synchronize()
        ref, ref_a = u.cpu().numpy().copy(), amax.cpu().numpy().copy()
        for replay in range(3):
            u.copy_(torch.from_numpy(U0))
            amax.zero_()
            rk.graph(dt, dx, amax)
            torch.cuda.synchronize()
            _ = torch.ones(16, device=dev).sum().item()       # eager work between replays
            rk.graph(dt, dx, amax)
            torch.cuda.synchronize()
            assert np.array_equal(u.cpu().numpy(), ref), replay
            assert np.array_equal(amax.cpu().numpy(), ref_a), replay
    finally:
        rk.close()


def _sod_l1_gpu(dev, nsub, t_end=0.2, cfl=0.4):
    U0, x = _sod_brick(nsub)
    n = 8
    dx = 1.0 / (n * nsub)
    u = torch.from_numpy(U0).to(dev)
    w, s = torch.empty_like(u), torch.empty_like(u)
    probe = torch.empty_like(u)
    amax = torch.zeros(nsub, dtype=torch.float64, device=dev)
    rk = hydroagg.RK3(hydroagg.brick(n, 6, (nsub, 1, 1), (1, 0, 0)), u, w, s)
    descs = hydroagg.subgrids(u, probe)
    t = 0.0
    try:
        while t < t_end - 1e-14:
            hydroagg.hydro_step(descs, 0.0, dx, amax)
            torch.cuda.synchronize()
            dt = min(cfl * dx / float(amax.max()), t_end - t)
            rk.step(dt, dx)
            t += dt
        torch.cuda.synchronize()
        U = u.cpu().numpy()
    finally:
        rk.close()
    rho = np.concatenate([U[k, 0, 3:11, 3:11, 3:11] for k in range(nsub)], axis=-1)
    assert np.max(np.abs(rho - rho[:1, :1, :])) < 1e-12        # every y-z line identical
    rho_ex, _, _ = riemann.sample((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 5.0 / 3.0, (x - 0.5) / t_end)
    return float(np.mean(np.abs(rho[0, 0] - rho_ex)))


def test_sod_converges_on_the_gpu(dev):
    errs = [_sod_l1_gpu(dev, nsub) for nsub in (4, 8, 16)]
    print(f"Sod L1(rho) at 32/64/128 cells: {errs}", flush=True)
    assert errs[0] / errs[1] >= 1.6 and errs[1] / errs[2] >= 1.6, errs
    assert errs[2] < 5e-3, errs
