"""Parity of the HIP path with the CPU oracle on the same seeded inputs.

Bar: per sub-grid and per field, max |U_gpu - U_oracle| / max |U_oracle| over
that sub-grid's interior cells <= 1e-12 (FP64 step; the two sides differ only
in rounding order), and the same pooled over the batch; amax relative error
<= 1e-13 per sub-grid.  Bitwise where the mathematics fixes the value
(uniform state, dt = 0, power-of-two scaling, batch independence)."""
import math

import numpy as np
import pytest

from paper_2210_06438_amd import hydroagg, workloads
from tests.gpu_util import ghost_mask, interior, normwise, normwise_each

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12
ATOL_AMAX = 1e-13


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def run_gpu(U, dt, dx, levels=None, each=False, dev="cuda:0"):
    """Step a [count, F, M, M, M] batch on the GPU; returns (u_out, amax)."""
    u_in = torch.from_numpy(np.ascontiguousarray(U)).to(dev)
    u_out = u_in.clone()
    amax = torch.zeros(U.shape[0], dtype=torch.float64, device=dev)
    descs = hydroagg.subgrids(u_in, u_out, levels=levels)
    (hydroagg.hydro_step_each if each else hydroagg.hydro_step)(descs, dt, dx, amax)
    torch.cuda.synchronize()
    return u_out.cpu().numpy(), amax.cpu().numpy()


def check(U, dt, dx, oracle_mod, levels=None, each=False):
    n = U.shape[2] - 6
    print(f"parity: count={U.shape[0]} n={n} F={U.shape[1]} dt={dt:.3e}", flush=True)
    ref, ref_amax = oracle_mod.step(U, dt, dx, levels=levels)
    got, amax = run_gpu(U, dt, dx, levels=levels, each=each)
    err = normwise(interior(got, n), interior(ref, n))
    assert np.all(err <= TOL), err
    each = normwise_each(interior(got, n), interior(ref, n))
    assert np.all(each <= TOL), (np.unravel_index(np.argmax(each), each.shape), each.max())
    rel = np.max(np.abs(amax - ref_amax) / ref_amax)
    assert rel <= ATOL_AMAX, rel
    g = ghost_mask(n)
    assert np.array_equal(got[:, :, g], U[:, :, g]), "ghost cells of u_out were written"
    return got, amax


def courant_dt(oracle_mod, U, dx, levels=None, cfl=0.4):
    _, a = oracle_mod.step(U, 0.0, dx, levels=levels)
    lv = np.zeros(len(a)) if levels is None else np.asarray(levels)
    return cfl * float(np.min(dx * 2.0 ** (-lv) / a))


def test_brick_c1(dev, oracle_mod):
    U = workloads.brick(seed=1)
    dx = 1 / 64
    check(U, courant_dt(oracle_mod, U, dx), dx, oracle_mod)


@pytest.mark.parametrize("n", [8, 12, 16])
@pytest.mark.parametrize("nf", [6, 11])
def test_random_smooth(dev, oracle_mod, n, nf):
    U = workloads.random_smooth(12, n=n, nfields=nf, seed=100 + n + nf)
    dx = 0.05
    check(U, courant_dt(oracle_mod, U, dx), dx, oracle_mod)


def test_small_batches_use_kernel_arguments(dev, oracle_mod):
    for count in (1, 3, 8, 9):
        U = workloads.random_smooth(count, n=8, nfields=11, seed=200 + count)
        check(U, 0.002, 0.05, oracle_mod)


def test_per_subgrid_launch_matches(dev, oracle_mod):
    U = workloads.random_smooth(10, n=12, nfields=11, seed=300)
    check(U, 0.002, 0.05, oracle_mod, each=True)


def test_polytrope_mix_with_levels(dev, oracle_mod):
    groups = workloads.polytrope(count=40, seed=3)
    for N, levels, U, _ in groups:
        dx = 0.5
        dt = courant_dt(oracle_mod, U, dx, levels=levels)
        check(U, dt, dx, oracle_mod, levels=levels)


def test_uniform_state_bitwise(dev):
    for n, nf in ((8, 6), (12, 11), (16, 11)):
        M = n + 6
        W = [1.3, 0.2, -0.4, 0.7, 2.1] + [0.3] * (nf - 5)
        e = W[4] / (5 / 3 - 1) + 0.5 * W[0] * (W[1] ** 2 + W[2] ** 2 + W[3] ** 2)
        Uc = np.array([W[0], W[0] * W[1], W[0] * W[2], W[0] * W[3], e] + W[5:])
        U = np.broadcast_to(Uc[None, :, None, None, None], (3, nf, M, M, M)).copy()
        got, amax = run_gpu(U, 0.01, 0.02)
        assert np.array_equal(got, U)
        c = math.sqrt(5 / 3 * 2.1 / 1.3)
        assert np.allclose(amax, 0.7 + c, rtol=1e-14, atol=0)


def test_dt_zero_and_scaling_bitwise(dev):
    U = workloads.random_smooth(6, n=8, nfields=11, seed=400)
    got0, _ = run_gpu(U, 0.0, 0.05)
    assert np.array_equal(got0, U)
    a, am = run_gpu(U, 0.003, 0.05, levels=[0, 1, 2, 0, 1, 2])
    b, bm = run_gpu(2.0 * U, 0.003, 0.05, levels=[0, 1, 2, 0, 1, 2])
    assert np.array_equal(interior(b, 8), 2.0 * interior(a, 8))
    assert np.array_equal(am, bm)
    c, cm = run_gpu(U, 0.006, 0.1, levels=[0, 1, 2, 0, 1, 2])
    assert np.array_equal(interior(c, 8), interior(a, 8)) and np.array_equal(cm, am)


def test_brick_conservation_on_gpu(dev):
    U = workloads.brick(seed=5)
    got, amax = run_gpu(U, 0.0, 1 / 64)
    dt = 0.4 / 64 / amax.max()
    got, _ = run_gpu(U, dt, 1 / 64)
    for f in range(U.shape[1]):
        before = math.fsum(interior(U, 8)[:, f].ravel())
        after = math.fsum(interior(got, 8)[:, f].ravel())
        scale = math.fsum(np.abs(interior(U, 8)[:, f]).ravel())
        assert abs(after - before) <= 1e-13 * scale


def test_batch_independence_bitwise(dev):
    """A sub-grid's result does not depend on the batch it runs in."""
    U8 = workloads.random_smooth(20, n=8, nfields=11, seed=500)
    U12 = workloads.random_smooth(5, n=12, nfields=11, seed=501)
    dt, dx = 0.002, 0.05
    alone = [run_gpu(U8[i:i + 1], dt, dx)[0][0] for i in (0, 7, 19)]
    batch, _ = run_gpu(U8, dt, dx)
    each, _ = run_gpu(U8, dt, dx, each=True)
    perm = np.random.default_rng(0).permutation(20)
    shuffled, _ = run_gpu(U8[perm], dt, dx)
    for k, i in enumerate((0, 7, 19)):
        assert np.array_equal(batch[i], alone[k])
    assert np.array_equal(batch, each)
    assert np.array_equal(shuffled, batch[perm])
    # mixed shapes in one call
    u8 = torch.from_numpy(U8).to(dev)
    u12 = torch.from_numpy(U12).to(dev)
    o8, o12 = u8.clone(), u12.clone()
    d = hydroagg.concat(hydroagg.subgrids(u12, o12), hydroagg.subgrids(u8, o8))
    hydroagg.hydro_step(d, dt, dx)
    torch.cuda.synchronize()
    assert np.array_equal(o8.cpu().numpy(), batch)
    ref12, _ = run_gpu(U12, dt, dx)
    assert np.array_equal(o12.cpu().numpy(), ref12)


def test_full_size_batch_sampled(dev, oracle_mod):
    """4096 sub-grids of 8^3 with 11 fields (the batching workload) in one
    aggregated call; a sample of sub-grids is checked against the oracle."""
    count = 4096
    print("full-size: generating 4096 x 8^3 x 11 fields", flush=True)
    U = workloads.random_smooth(count, n=8, nfields=11, seed=2)
    u_in = torch.from_numpy(U).to(dev)
    u_out = u_in.clone()
    amax = torch.zeros(count, dtype=torch.float64, device=dev)
    d = hydroagg.subgrids(u_in, u_out)
    hydroagg.hydro_step(d, 0.0, 1 / 64, amax)
    torch.cuda.synchronize()
    dt = 0.4 / 64 / float(amax.max())
    hydroagg.hydro_step(d, dt, 1 / 64, amax)
    torch.cuda.synchronize()
    sample = np.unique(np.r_[0, count - 1, np.random.default_rng(1).integers(0, count, 14)])
    got = u_out[torch.from_numpy(sample).to(dev)].cpu().numpy()
    ref, ref_amax = oracle_mod.step(U[sample], dt, 1 / 64)
    assert np.all(normwise_each(interior(got, 8), interior(ref, 8)) <= TOL)
    a = amax.cpu().numpy()[sample]
    assert np.max(np.abs(a - ref_amax) / ref_amax) <= ATOL_AMAX


def test_x_only_data_has_no_transverse_update_on_gpu(dev, oracle_mod):
    from tests.test_oracle_pins import x_only_block
    for n, nf in ((8, 11), (12, 6), (16, 11)):
        U = np.stack([x_only_block(n, nf, seed=n + nf + s) for s in range(3)])
        got, amax = run_gpu(U, 0.002, 0.05)
        I = interior(got, n)
        assert np.array_equal(I, np.broadcast_to(I[:, :, :1, :1, :], I.shape))
        assert not I[:, 2].any() and not I[:, 3].any()
        check(U, 0.002, 0.05, oracle_mod)


def _step_layouts(U, levels, dt, dx, dev, each=False):
    """Step U once with stored-layout and once with interior-only outputs."""
    count, nf, M = U.shape[0], U.shape[1], U.shape[2]
    n = M - 6
    u_in = torch.from_numpy(U).to(dev)
    a = u_in.clone()
    b = torch.full((count, nf, n, n, n), float("nan"), dtype=torch.float64, device=dev)
    am_a = torch.zeros(count, dtype=torch.float64, device=dev)
    am_b = torch.zeros(count, dtype=torch.float64, device=dev)
    step = hydroagg.hydro_step_each if each else hydroagg.hydro_step
    step(hydroagg.subgrids(u_in, a, levels=levels), dt, dx, am_a)
    step(hydroagg.subgrids(u_in, b, levels=levels), dt, dx, am_b)
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy(), am_a.cpu().numpy(), am_b.cpu().numpy()


@pytest.mark.parametrize("n,nf,count,each", [(8, 11, 37, False), (8, 6, 5, False), (12, 11, 11, False),
                                             (12, 6, 3, False), (16, 11, 9, False),
                                             (16, 6, 2, True), (8, 11, 3, True)])
def test_interior_layout_matches_stored_layout(dev, n, nf, count, each):
    U = workloads.random_smooth(count, n=n, nfields=nf, seed=700 + n + nf + count)
    levels = [s % 3 for s in range(count)]
    print(f"layouts: n={n} F={nf} count={count} each={each}", flush=True)
    a, b, am_a, am_b = _step_layouts(U, levels, 2e-3, 0.05, dev, each=each)
    assert np.array_equal(interior(a, n), b)           # every element written, bitwise
    assert np.array_equal(am_a, am_b)
    g = ghost_mask(n)
    assert np.array_equal(a[:, :, g], U[:, :, g])


def test_layouts_mixed_in_one_batch(dev):
    n, nf, count = 8, 11, 24
    U = workloads.random_smooth(count, n=n, nfields=nf, seed=777)
    u_in = torch.from_numpy(U).to(dev)
    a = u_in[:12].clone()
    b = torch.zeros((12, nf, n, n, n), dtype=torch.float64, device=dev)
    batch = hydroagg.concat(hydroagg.subgrids(u_in[:12], a), hydroagg.subgrids(u_in[12:], b))
    amax = torch.zeros(count, dtype=torch.float64, device=dev)
    hydroagg.hydro_step(batch, 1e-3, 0.05, amax)
    torch.cuda.synchronize()
    ref, ref_a = run_gpu(U, 1e-3, 0.05)
    assert np.array_equal(a.cpu().numpy(), ref[:12])
    assert np.array_equal(b.cpu().numpy(), interior(ref[12:], n))
    assert np.array_equal(amax.cpu().numpy(), ref_a)


@pytest.mark.parametrize("n,nf,count", [(8, 11, 21), (8, 6, 3), (12, 11, 10), (12, 6, 4),
                                        (16, 11, 9), (16, 6, 2)])
def test_tiles_are_bitwise_equivalent(dev, oracle_mod, n, nf, count):
    """8^3 and 4^3 tiles compute every face from the same cells: both match
    the oracle, and each other far inside the parity tolerance (the two
    kernels are compiled separately, so contractions may differ in the last
    bits)."""
    U = workloads.random_smooth(count, n=n, nfields=nf, seed=900 + n + nf + count)
    levels = [s % 2 for s in range(count)]
    before = hydroagg.get_tile(n, nf)
    out = {}
    try:
        for tile in (8, 4):
            hydroagg.set_tile(n, nf, tile)
            print(f"tiles: n={n} F={nf} count={count} tile={tile}", flush=True)
            out[tile] = check(U, 2e-3, 0.05, oracle_mod, levels=levels)
    finally:
        hydroagg.set_tile(n, nf, before)
    diff = normwise_each(interior(out[4][0], n), interior(out[8][0], n))
    da = np.max(np.abs(out[4][1] - out[8][1]) / out[8][1])
    print(f"tile 4 vs 8: normwise {diff.max():.2e}, amax {da:.2e}", flush=True)
    assert diff.max() <= 1e-13 and da <= 1e-14


def test_plan_recaptures_after_a_tile_change(dev):
    n, nf, count = 8, 11, 16
    U = workloads.random_smooth(count, n=n, nfields=nf, seed=950)
    u_in = torch.from_numpy(U).to(dev)
    u_out = u_in.clone()
    amax = torch.zeros(count, dtype=torch.float64, device=dev)
    plan = hydroagg.Plan(hydroagg.subgrids(u_in, u_out))
    stream = torch.cuda.current_stream()
    before = hydroagg.get_tile(n, nf)
    try:
        plan.graph(1e-3, 0.05, amax, stream)
        torch.cuda.synchronize()
        ref = u_out.cpu().numpy().copy()
        u_out.zero_()
        hydroagg.set_tile(n, nf, 4 if before == 8 else 8)
        plan.graph(1e-3, 0.05, amax, stream)
        torch.cuda.synchronize()
        got = u_out.cpu().numpy()
    finally:
        hydroagg.set_tile(n, nf, before)
        plan.close()
    assert normwise_each(interior(got, n), interior(ref, n)).max() <= 1e-13
    assert not np.array_equal(interior(got, n), np.zeros_like(interior(got, n)))


def test_batch_larger_than_a_staging_slot(dev, oracle_mod):
    """66000 sub-grids (two descriptor-staging chunks of at most 65536):
    1031 distinct ones, replicated on the device.  The distinct ones match
    the oracle, and every copy is bitwise its original, wherever it sits."""
    uniq = workloads.random_smooth(1031, n=8, nfields=6, seed=1200)
    count = 66000
    print(f"large batch: count={count} n=8 F=6", flush=True)
    idx = torch.arange(count, device=dev) % 1031
    u_in = torch.from_numpy(uniq).to(dev)[idx].contiguous()
    u_out = u_in.clone()
    amax = torch.zeros(count, dtype=torch.float64, device=dev)
    dt, dx = 1e-3, 1.0 / 64
    hydroagg.hydro_step(hydroagg.subgrids(u_in, u_out), dt, dx, amax)
    torch.cuda.synchronize()
    first = u_out[:1031]
    assert torch.equal(u_out, first[idx]) and torch.equal(amax, amax[:1031][idx])
    ref, ref_amax = oracle_mod.step(uniq, dt, dx)
    got = first.cpu().numpy()
    assert np.all(normwise_each(interior(got, 8), interior(ref, 8)) <= TOL)
    assert np.max(np.abs(amax[:1031].cpu().numpy() - ref_amax) / ref_amax) <= ATOL_AMAX
    del u_in, u_out


MIXES = {
    # every class small: the graph runs them in sequence
    "six_small_classes": [((8, 6), 20), ((8, 11), 20), ((12, 6), 20), ((12, 11), 20),
                          ((16, 6), 20), ((16, 11), 20)],
    # two classes of >= 1024 work-groups (one becomes a side branch) and two
    # small ones of one field count (one multi-class launch) beside them
    "two_large_classes": [((8, 6), 1024), ((16, 6), 128), ((12, 11), 5), ((8, 11), 3)],
    # small classes of one field count: one multi-class launch from the
    # plan's device table (the eager step passes them in the arguments)
    "three_small_one_field_count": [((8, 11), 5), ((12, 11), 4), ((16, 11), 3)],
    # one large class alone (no branch: it is the only one) beside one
    # multi-class launch of two small ones
    "one_large_two_small": [((8, 11), 1100), ((12, 11), 5), ((16, 11), 3)],
}


@pytest.mark.parametrize("mix", sorted(MIXES))
def test_plan_graph_matches_eager_step(dev, mix):
    """A plan's graph (classes in sequence, or large classes as concurrent
    branches) gives, on every replay with eager work between replays, bitwise
    the eager hydro_step result: outputs and amax."""
    parts = []
    before = {(n, nf): hydroagg.get_tile(n, nf) for (n, nf), _ in MIXES[mix]}
    for k, ((n, nf), cnt) in enumerate(MIXES[mix]):
        U = workloads.random_smooth(cnt, n=n, nfields=nf, seed=1300 + k)
        u_in = torch.from_numpy(U).to(dev)
        parts.append((u_in, u_in.clone(), u_in.clone()))
    count = sum(c for _, c in MIXES[mix])
    graph_descs = hydroagg.concat(*[hydroagg.subgrids(a, b) for a, b, _ in parts])
    eager_descs = hydroagg.concat(*[hydroagg.subgrids(a, c) for a, _, c in parts])
    amax_g = torch.zeros(count, dtype=torch.float64, device=dev)
    amax_e = torch.zeros(count, dtype=torch.float64, device=dev)
    dt, dx = 2e-3, 0.05
    print(f"plan graph: {mix}", flush=True)
    plan = None
    try:
        for (n, nf), _ in MIXES[mix]:
            if mix in ("two_large_classes", "one_large_two_small"):
                hydroagg.set_tile(n, nf, 8)   # 8^3 blocks: >= 1024 work-groups per large class
        hydroagg.hydro_step(eager_descs, dt, dx, amax_e)
        torch.cuda.synchronize()
        plan = hydroagg.Plan(graph_descs)
        stream = torch.cuda.current_stream()
        for replay in range(3):
            for _, b, _ in parts:
                b.fill_(-1.0)
            amax_g.zero_()
            plan.graph(dt, dx, amax_g, stream)
            torch.cuda.synchronize()
            for _, b, c in parts:
                i = (slice(None), slice(None), slice(3, -3), slice(3, -3), slice(3, -3))
                assert torch.equal(b[i], c[i]), f"replay {replay}"
            assert torch.equal(amax_g, amax_e), f"replay {replay}"
    finally:
        for (n, nf), t in before.items():
            hydroagg.set_tile(n, nf, t)
        if plan is not None:
            plan.close()


TILE_SETS = {"default": None, "all_4": 4, "all_8": 8}


def _with_tiles(tiles, fn):
    keys = [(n, nf) for n in (8, 12, 16) for nf in (6, 11)]
    before = {k: hydroagg.get_tile(*k) for k in keys}
    try:
        if tiles is not None:
            for k in keys:
                hydroagg.set_tile(*k, tiles)
        return fn()
    finally:
        for k, t in before.items():
            hydroagg.set_tile(*k, t)


MIXED_COUNTS = {"arguments": {8: 3, 12: 2, 16: 2}, "table": {8: 13, 12: 10, 16: 9}}


@pytest.mark.parametrize("tiles", sorted(TILE_SETS))
@pytest.mark.parametrize("nf", [6, 11])
@pytest.mark.parametrize("form", sorted(MIXED_COUNTS))
def test_mixed_batch_is_one_launch_bitwise_alone(dev, oracle_mod, tiles, nf, form):
    """A batch of 8^3, 12^3 and 16^3 sub-grids of one field count is one
    multi-class launch (descriptors in the kernel arguments up to 8 per
    class, else in a device table); every sub-grid is bitwise what it is
    stepped alone (its class kernel) and matches the oracle."""
    counts = MIXED_COUNTS[form]
    dt, dx = 2e-3, 0.05
    print(f"mixed: form={form} F={nf} tiles={tiles}", flush=True)

    def run():
        out = {}
        parts = {}
        for n, c in counts.items():
            U = workloads.random_smooth(c, n=n, nfields=nf, seed=1400 + n + nf)
            t = torch.from_numpy(U).to(dev)
            parts[n] = (U, t, t.clone())
        amax = torch.zeros(sum(counts.values()), dtype=torch.float64, device=dev)
        hydroagg.hydro_step(hydroagg.concat(*[hydroagg.subgrids(a, b) for _, a, b in parts.values()]),
                            dt, dx, amax)
        torch.cuda.synchronize()
        k = 0
        for n, (U, a, b) in parts.items():
            got = b.cpu().numpy()
            ref, ref_a = run_gpu(U, dt, dx, each=True)   # one launch per sub-grid
            assert np.array_equal(interior(got, n), interior(ref, n)), n
            assert np.array_equal(amax.cpu().numpy()[k:k + len(U)], ref_a), n
            o, oa = oracle_mod.step(U, dt, dx)
            assert np.all(normwise_each(interior(got, n), interior(o, n)) <= TOL)
            k += len(U)
    _with_tiles(TILE_SETS[tiles], run)


def test_concurrent_host_threads_share_the_descriptor_ring(dev):
    """Four host threads, each on its own stream, issue 24 table-path steps
    each (96 calls in flight against 8 staging slots): every result is
    bitwise the single-threaded one."""
    import threading
    U = workloads.random_smooth(40, n=8, nfields=11, seed=1500)
    dt, dx = 1e-3, 0.05
    ref, ref_a = run_gpu(U, dt, dx)
    u_in = torch.from_numpy(U).to(dev)
    outs = [torch.zeros_like(u_in) for _ in range(4)]
    amaxs = [torch.zeros(40, dtype=torch.float64, device=dev) for _ in range(4)]
    descs = [hydroagg.subgrids(u_in, o) for o in outs]
    streams = [torch.cuda.Stream() for _ in range(4)]
    errors = []

    def work(k):
        try:
            for _ in range(24):
                hydroagg.hydro_step(descs[k], dt, dx, amaxs[k], streams[k])
        except Exception as e:          # noqa: BLE001 - reported below
            errors.append(e)

    threads = [threading.Thread(target=work, args=(k,)) for k in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize()
    assert not errors, errors
    for k in range(4):
        assert np.array_equal(interior(outs[k].cpu().numpy(), 8), interior(ref, 8)), k
        assert np.array_equal(amaxs[k].cpu().numpy(), ref_a), k
