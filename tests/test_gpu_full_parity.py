"""Parity of every sub-grid of the two throughput workloads with the CPU
oracle, through the launch the benchmark times (a plan's hipGraph).

* 4096 independent 8^3 sub-grids, 11 FP64 fields (random smooth state), one
  graph launch of the aggregated kernel, with each tile.
* 3000 polytrope sub-grids of edges 8/12/16, 11 fields, random octree levels,
  one graph launch holding one multi-class kernel, with each tile set.  About
  60% of these sub-grids hold only the 1e-10 atmosphere.

Bar: per sub-grid AND per field, max |U_gpu - U_oracle| / max |U_oracle| over
that sub-grid's interior <= 1e-12 (the pooled metric over the whole batch is
checked too, but it cannot see errors in sub-grids whose values are far
below the batch maximum); amax relative error <= 1e-13 per sub-grid; ghost
cells of u_out never written.  Each replay starts from NaN-filled outputs.
"""
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


def _check_group(tag, got, ref, amax, ref_amax, n):
    each = normwise_each(interior(got, n), interior(ref, n))
    worst = np.unravel_index(np.argmax(each), each.shape)
    print(f"{tag}: n={n} count={got.shape[0]} worst per-sub-grid normwise {each.max():.2e} "
          f"(sub-grid {worst[0]}, field {worst[1]}); pooled {normwise(interior(got, n), interior(ref, n)).max():.2e}",
          flush=True)
    assert np.all(each <= TOL), (tag, worst, each.max())
    assert np.all(normwise(interior(got, n), interior(ref, n)) <= TOL)
    rel = np.abs(amax - ref_amax) / ref_amax
    assert np.all(rel <= TOL_AMAX), (tag, int(np.argmax(rel)), rel.max())
    ghosts = got.copy()
    ghosts[..., 3:3 + n, 3:3 + n, 3:3 + n] = np.nan
    assert np.all(np.isnan(ghosts)), f"{tag}: ghost cells of u_out were written"


def _set_tiles(pairs, tile):
    for n, nf in pairs:
        hydroagg.set_tile(n, nf, tile)


def test_random_smooth_4096_every_subgrid_through_the_graph(dev, oracle_mod):
    count, n, nf, dx = 4096, 8, 11, 1.0 / 64
    print("C2 full: generating 4096 x 8^3 x 11 fields", flush=True)
    U = workloads.random_smooth(count, n=n, nfields=nf, seed=2)
    u_in = torch.from_numpy(U).to(dev)
    u_out = u_in.clone()
    amax = torch.zeros(count, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    plan = hydroagg.Plan(hydroagg.subgrids(u_in, u_out))
    before = hydroagg.get_tile(n, nf)
    try:
        plan.step(0.0, dx, amax, stream)
        torch.cuda.synchronize()
        dt = 0.4 * dx / float(amax.max())
        ref, ref_amax = oracle_mod.step(U, dt, dx, nthreads=oracle_threads())
        for tile in (8, 4):
            hydroagg.set_tile(n, nf, tile)
            for replay in range(2):
                print(f"C2 full: tile {tile}, replay {replay}", flush=True)
                u_out.fill_(float("nan"))
                amax.fill_(float("nan"))
                plan.graph(dt, dx, amax, stream)
                torch.cuda.synchronize()
                _check_group(f"C2 tile {tile} replay {replay}", u_out.cpu().numpy(), ref,
                             amax.cpu().numpy(), ref_amax, n)
    finally:
        hydroagg.set_tile(n, nf, before)
        plan.close()


TILE_SETS = {"default": None, "all_4": 4, "all_8": 8}


def test_polytrope_3000_every_subgrid_through_one_graph_launch(dev, oracle_mod):
    dx, nf = 0.5, 11
    print("C3 full: generating 3000 polytrope sub-grids", flush=True)
    groups = workloads.polytrope(count=3000, seed=3)
    atm = sum(int(np.sum(np.all(U[:, 0] <= workloads.ATMOSPHERE, axis=(1, 2, 3))))
              for _, _, U, _ in groups)
    print(f"C3 full: {atm} of 3000 sub-grids are atmosphere only", flush=True)
    parts = []
    for N, levels, U, _ in groups:
        t = torch.from_numpy(U).to(dev)
        parts.append((N, levels, U, t, torch.empty_like(t)))
    count = sum(U.shape[0] for _, _, U, _, _ in parts)
    amax = torch.zeros(count, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    plan = hydroagg.Plan(hydroagg.concat(*[hydroagg.subgrids(a, b, levels=lv)
                                           for _, lv, _, a, b in parts]))
    pairs = [(N, nf) for N in (8, 12, 16)]
    before = {p: hydroagg.get_tile(*p) for p in pairs}
    try:
        plan.step(0.0, dx, amax, stream)
        torch.cuda.synchronize()
        lv = np.concatenate([l for _, l, _, _, _ in parts]).astype(np.float64)
        dt = 0.4 * float(np.min(dx * 2.0 ** (-lv) / amax.cpu().numpy()))
        refs = [oracle_mod.step(U, dt, dx, levels=l, nthreads=oracle_threads())
                for _, l, U, _, _ in parts]
        for name, tile in TILE_SETS.items():
            if tile is None:
                for p, t in before.items():
                    hydroagg.set_tile(*p, t)
            else:
                _set_tiles(pairs, tile)
            for replay in range(2):
                print(f"C3 full: tiles {name}, replay {replay}", flush=True)
                for _, _, _, _, b in parts:
                    b.fill_(float("nan"))
                amax.fill_(float("nan"))
                plan.graph(dt, dx, amax, stream)
                torch.cuda.synchronize()
                am = amax.cpu().numpy()
                k = 0
                for (N, _, U, _, b), (ref, ref_amax) in zip(parts, refs):
                    _check_group(f"C3 tiles {name} replay {replay}", b.cpu().numpy(), ref,
                                 am[k:k + U.shape[0]], ref_amax, N)
                    k += U.shape[0]
    finally:
        for p, t in before.items():
            hydroagg.set_tile(*p, t)
        plan.close()
