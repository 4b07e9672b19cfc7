"""Aggregator and serving loop on the GPU.  Every task's result must be
bitwise identical to the same sub-grid stepped alone by hydro_step, whatever
batch, width, stream or admission order it ran in (batch independence)."""
import numpy as np
import pytest

from paper_2210_06438_amd import hydroagg, workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def alone(U, dt, dx, levels=None):
    """Reference: hydro_step on each sub-grid separately."""
    outs, amaxs = [], []
    for i in range(U.shape[0]):
        u_in = torch.from_numpy(np.ascontiguousarray(U[i:i + 1])).cuda()
        u_out = u_in.clone()
        am = torch.zeros(1, dtype=torch.float64, device="cuda")
        hydroagg.hydro_step(hydroagg.subgrids(u_in, u_out, levels=None if levels is None else [levels[i]]),
                            dt, dx, am)
        torch.cuda.synchronize()
        outs.append(u_out.cpu().numpy()[0])
        amaxs.append(float(am.cpu()[0]))
    return outs, amaxs


@pytest.mark.parametrize("width,streams,idle", [(1, 1, False), (4, 2, True), (64, 2, True), (5, 1, False)])
def test_aggregator_results_match_alone(dev, width, streams, idle):
    print(f"agg: width={width} streams={streams} idle={idle}", flush=True)
    U8 = workloads.random_smooth(9, n=8, nfields=11, seed=600)
    U12 = workloads.random_smooth(4, n=12, nfields=11, seed=601)
    dt, dx = 0.002, 0.05
    r8, a8 = alone(U8, dt, dx)
    r12, a12 = alone(U12, dt, dx)
    u8 = torch.from_numpy(U8).to(dev)
    u12 = torch.from_numpy(U12).to(dev)
    o8, o12 = u8.clone(), u12.clone()
    d8, _ = hydroagg.subgrids(u8, o8)
    d12, _ = hydroagg.subgrids(u12, o12)
    agg = hydroagg.Aggregator(width, timeout_us=-1.0, n_streams=streams, flush_when_idle=idle)
    tickets = []
    order = [("8", i) for i in range(9)] + [("12", i) for i in range(4)]
    np.random.default_rng(width).shuffle(order)
    for kind, i in order:
        tickets.append((kind, i, agg.submit((d8 if kind == "8" else d12)[i], dt, dx)))
    agg.flush()
    got = {}
    for kind, i, t in tickets:
        got[(kind, i)] = agg.wait(t)
    st = agg.stats()
    agg.close()
    torch.cuda.synchronize()
    assert st["launched"] == 13 and st["submitted"] == 13
    if width == 1:
        assert st["batches"] == 13
    O8, O12 = o8.cpu().numpy(), o12.cpu().numpy()
    for i in range(9):
        assert np.array_equal(O8[i], r8[i]) and got[("8", i)] == a8[i]
    for i in range(4):
        assert np.array_equal(O12[i], r12[i]) and got[("12", i)] == a12[i]


def test_aggregator_byte_budget(dev):
    U = workloads.random_smooth(10, n=8, nfields=6, seed=610)
    dt, dx = 0.002, 0.05
    ref, ref_a = alone(U, dt, dx)
    u = torch.from_numpy(U).to(dev)
    o = u.clone()
    d, _ = hydroagg.subgrids(u, o)
    per = U[0].nbytes
    agg = hydroagg.Aggregator(2, timeout_us=-1.0, n_streams=1, hbm_budget_bytes=3 * per,
                              flush_when_idle=False)
    tickets, refused = [], 0
    for i in range(10):
        while True:
            t = agg.try_submit(d[i], dt, dx)
            if t is not None:
                tickets.append(t)
                break
            refused += 1
            agg.flush()
            agg.progress()
    amax = [agg.wait(t) for t in tickets]
    st = agg.stats()
    agg.close()
    torch.cuda.synchronize()
    assert refused > 0 and st["refused"] == refused
    assert np.array_equal(o.cpu().numpy(), np.stack(ref)) and amax == ref_a


def test_aggregator_errors(dev):
    with pytest.raises(hydroagg.HydroError):
        hydroagg.Aggregator(0)
    with pytest.raises(hydroagg.HydroError):
        hydroagg.Aggregator(4, n_streams=129)
    agg = hydroagg.Aggregator(4)
    with pytest.raises(hydroagg.HydroError):
        agg.poll(12345)
    with pytest.raises(hydroagg.HydroError):
        agg.wait(12345)
    agg.close()


def _pool(dev, count=24, seed=620):
    groups = workloads.polytrope(count=count, seed=seed)
    tensors, descs, host = [], [], []
    for N, levels, U, _ in groups:
        t = torch.from_numpy(U).to(dev)
        tensors.append(t)
        descs.append(hydroagg.subgrids(t, t.clone(), levels=levels))
        host.append((N, levels, U))
    pool = hydroagg.concat(*descs)
    # flatten the host side in the same order
    Us, Ls, Ns = [], [], []
    for N, levels, U in host:
        for i in range(U.shape[0]):
            Us.append(U[i])
            Ls.append(int(levels[i]))
            Ns.append(N)
    return pool, tensors, Us, Ls, Ns


@pytest.mark.parametrize("layout", [hydroagg.OUT_STORED, hydroagg.OUT_INTERIOR])
def test_serving_loop_results_match_alone(dev, layout):
    pool, keep, Us, Ls, Ns = _pool(dev)
    rng = np.random.default_rng(7)
    ntask = 90
    task = rng.integers(0, len(Us), ntask).astype(np.int32)
    arrival = np.cumsum(rng.exponential(50.0, ntask))          # 20k tasks/s
    dx = 0.5
    dt = 1e-4
    inner_only = layout == hydroagg.OUT_INTERIOR
    sizes = {N: (N if inner_only else N + 6) ** 3 for N in (8, 12, 16)}
    counts = {N: int(np.sum(np.array([Ns[s] for s in task]) == N)) for N in (8, 12, 16)}
    arenas = []
    for N in (8, 12, 16):
        k = counts[N]
        arenas.append((torch.zeros(max(k, 1) * 11 * sizes[N], dtype=torch.float64, device=dev), k))
    lat, am, slabs, st = hydroagg.serve_run(pool, task, arrival, nfields=11, dt=dt, dx=dx,
                                            slab_arenas=arenas, max_width=16, timeout_us=50.0,
                                            n_streams=2, keep_slabs=True, want_slabs=True,
                                            out_layout=layout)
    torch.cuda.synchronize()
    assert st["agg"]["launched"] == ntask and np.all(lat > 0)
    # compare each task's slab with the sub-grid stepped alone
    base = {N: arenas[e][0].data_ptr() for e, N in enumerate((8, 12, 16))}
    arena_host = {N: arenas[e][0].cpu().numpy() for e, N in enumerate((8, 12, 16))}
    checked = 0
    for i in range(ntask):
        s = int(task[i])
        N = Ns[s]
        E = N if inner_only else N + 6
        off = (int(slabs[i]) - base[N]) // 8
        out = arena_host[N][off:off + 11 * E ** 3].reshape(11, E, E, E)
        ref, ref_a = alone(Us[s][None], dt, dx, levels=[Ls[s]])
        inner = (slice(None), slice(3, 3 + N), slice(3, 3 + N), slice(3, 3 + N))
        got = out if inner_only else out[inner]
        assert np.array_equal(got, ref[0][inner]), i
        assert am[i] == ref_a[0]
        checked += 1
    assert checked == ntask


def test_serving_loop_admission_bound(dev):
    pool, keep, Us, Ls, Ns = _pool(dev, count=16, seed=630)
    rng = np.random.default_rng(8)
    ntask = 600
    task = rng.integers(0, len(Us), ntask).astype(np.int32)
    arrival = np.cumsum(rng.exponential(5.0, ntask))            # 200k tasks/s: overload
    sizes = {8: 14 ** 3, 12: 18 ** 3, 16: 22 ** 3}
    arenas = [(torch.zeros(4 * 11 * sizes[N], dtype=torch.float64, device=dev), 4) for N in (8, 12, 16)]
    lat, am, _, st = hydroagg.serve_run(pool, task, arrival, nfields=11, dt=1e-4, dx=0.5,
                                        slab_arenas=arenas, max_width=8, timeout_us=50.0,
                                        n_streams=2)
    torch.cuda.synchronize()
    assert st["agg"]["launched"] == ntask and st["max_live"] <= 12
    assert st["slab_waits"] > 0 and np.all(lat > 0) and np.all(am > 0)


def test_tile_sweep_chooses_and_applies(dev):
    from paper_2210_06438_amd import tune
    before = {(n, f): hydroagg.get_tile(n, f) for n in (8, 12, 16) for f in (6, 11)}
    try:
        recs, best = tune.tile_sweep(count=16, reps=2, warmup=1, dev=dev, apply=False)
        assert set(best) == set(before) and all(t in (4, 8) for t in best.values())
        assert len(recs) == 12 and all(r["us_per_step"] > 0 for r in recs)
        assert {k: hydroagg.get_tile(*k) for k in before} == before      # apply=False restores
        recs, best = tune.tile_sweep(count=16, reps=2, warmup=1, edges=(12,), fields=(11,),
                                     dev=dev, apply=True)
        assert hydroagg.get_tile(12, 11) == best[(12, 11)]
    finally:
        for (n, f), t in before.items():
            hydroagg.set_tile(n, f, t)


@pytest.mark.parametrize("tiles", [None, 4, 8])
def test_aggregator_mixed_batch_table_form(dev, tiles):
    """One aggregated batch of more than 8 sub-grids per class (8^3, 12^3,
    16^3; descriptors in a device table, one multi-class launch): every task
    is bitwise what it is stepped alone."""
    keys = [(n, 11) for n in (8, 12, 16)]
    before = {k: hydroagg.get_tile(*k) for k in keys}
    print(f"agg mixed table: tiles={tiles}", flush=True)
    try:
        if tiles is not None:
            for k in keys:
                hydroagg.set_tile(*k, tiles)
        dt, dx = 0.002, 0.05
        Us = {n: workloads.random_smooth(c, n=n, nfields=11, seed=1500 + n)
              for n, c in ((8, 10), (12, 9), (16, 9))}
        ins = {n: torch.from_numpy(U).to(dev) for n, U in Us.items()}
        outs = {n: t.clone() for n, t in ins.items()}
        descs = {n: hydroagg.subgrids(ins[n], outs[n])[0] for n in Us}
        agg = hydroagg.Aggregator(64, timeout_us=-1.0, n_streams=1, flush_when_idle=False)
        tickets = [(n, i, agg.submit(descs[n][i], dt, dx)) for n in Us for i in range(len(Us[n]))]
        agg.flush()
        got = {(n, i): agg.wait(t) for n, i, t in tickets}
        st = agg.stats()
        agg.close()
        torch.cuda.synchronize()
        assert st["batches"] == 1 and st["launched"] == 28
        for n, U in Us.items():
            ref, ref_a = alone(U, dt, dx)
            O = outs[n].cpu().numpy()
            for i in range(len(U)):
                assert np.array_equal(O[i], ref[i]) and got[(n, i)] == ref_a[i], (n, i)
    finally:
        for k, t in before.items():
            hydroagg.set_tile(*k, t)


def test_aggregator_batch_of_two_field_counts(dev):
    """One batch holding sub-grids of both field counts and all three edges
    (one multi-class launch per field count, amax partials of both): every
    task is bitwise what it is stepped alone."""
    dt, dx = 0.002, 0.05
    shapes = [(8, 6, 3), (12, 6, 2), (16, 6, 2), (8, 11, 4), (12, 11, 2), (16, 11, 9)]
    Us = {(n, nf): workloads.random_smooth(c, n=n, nfields=nf, seed=1600 + n + nf)
          for n, nf, c in shapes}
    ins = {k: torch.from_numpy(U).to(dev) for k, U in Us.items()}
    outs = {k: t.clone() for k, t in ins.items()}
    descs = {k: hydroagg.subgrids(ins[k], outs[k])[0] for k in Us}
    print("agg two field counts", flush=True)
    agg = hydroagg.Aggregator(64, timeout_us=-1.0, n_streams=1, flush_when_idle=False)
    order = [(k, i) for k in Us for i in range(len(Us[k]))]
    np.random.default_rng(3).shuffle(order)
    tickets = [(k, i, agg.submit(descs[k][i], dt, dx)) for k, i in order]
    agg.flush()
    got = {(k, i): agg.wait(t) for k, i, t in tickets}
    st = agg.stats()
    agg.close()
    torch.cuda.synchronize()
    assert st["batches"] == 1 and st["launched"] == len(order)
    for k, U in Us.items():
        ref, ref_a = alone(U, dt, dx)
        O = outs[k].cpu().numpy()
        for i in range(len(U)):
            assert np.array_equal(O[i], ref[i]) and got[(k, i)] == ref_a[i], (k, i)
