"""Aggregation regions on the GPU (paper Section V-D): host threads that
each step one sub-grid through a region -- a descriptor chunk and an amax
chunk of shared team buffers, one upload, one launch of the library's step
kernel and one download per team -- get bitwise the result and amax of
hydro_step; the first task holds its team open so that a full team queues
behind it.  The auxiliary kernel (a x + b y per member) runs the same way.
The library's task driver steps a batch from many threads through a region
and as one launch per task, both bitwise hydro_step."""
import ctypes
import threading
import time

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


def _run_threads(fns, first_hold=None, region=None, seated_tasks=0):
    """Start fns[0]; once it is seated start the rest; release it when the
    region has seated `seated_tasks` tasks."""
    errs = []

    def wrap(f):
        def g():
            try:
                f()
            except Exception as e:   # reported after the join
                errs.append(e)
        return g
    ts = [threading.Thread(target=wrap(f)) for f in fns]
    ts[0].start()
    if first_hold is not None:
        assert first_hold["seated"].wait(30)
    for t in ts[1:]:
        t.start()
    if first_hold is not None:
        t0 = time.time()
        while region.stats()["tasks"] < seated_tasks and time.time() - t0 < 30:
            time.sleep(0.001)
        first_hold["release"].set()
    for t in ts:
        t.join(60)
        assert not t.is_alive()
    assert not errs, errs


def test_threads_step_subgrids_through_a_region(dev):
    count, nf, dt, dx = 24, 11, 0.002, 0.05
    print("region: 24 threads, max team 8", flush=True)
    U = workloads.random_smooth(count, n=8, nfields=nf, seed=811)
    u_in = torch.from_numpy(U).to(dev)
    ref_out = torch.full((count, nf, 8, 8, 8), float("nan"), dtype=torch.float64, device=dev)
    ref_amax = torch.zeros(count, dtype=torch.float64, device=dev)
    hydroagg.hydro_step(hydroagg.subgrids(u_in, ref_out), dt, dx, ref_amax)
    torch.cuda.synchronize()
    out = torch.full_like(ref_out, float("nan"))
    descs, _ = hydroagg.subgrids(u_in, out)
    region = hydroagg.Region(max_team=8, n_streams=1, arena_bytes=1 << 16)
    kernel = hydroagg.region_kernel(hydroagg.REGION_STEP8_F11)
    amax = [None] * count
    teams = [None] * count
    hold = {"seated": threading.Event(), "release": threading.Event()}

    def task(i):
        def run():
            t = region.enter()
            teams[i] = (t.id, t.index, t.size)
            if i == 0:
                hold["seated"].set()
                assert hold["release"].wait(30)
            bd, hd, _ = region.alloc(t, 32)
            ba, ha, _ = region.alloc(t, 8)
            ctypes.memmove(hd, ctypes.byref(descs[i]), 32)
            region.upload(t, bd)
            base_d, stride = region.buffer(t, bd)
            base_a, _ = region.buffer(t, ba)
            assert stride == 32
            region.launch(t, kernel, 1, 192, [ctypes.c_void_p(base_d), ctypes.c_int32(t.size),
                                              ctypes.c_double(dt), ctypes.c_double(dx),
                                              ctypes.c_void_p(base_a)])
            region.download(t, ba)
            region.wait(t)
            amax[i] = ctypes.c_double.from_address(ha).value   # valid until leave
            region.leave(t)
        return run
    _run_threads([task(i) for i in range(count)], hold, region, seated_tasks=9)
    st = region.stats()
    region.close()
    print(f"region stats: {st}", flush=True)
    assert st["tasks"] == count and st["launches"] == st["teams"] == st["uploads"]
    assert st["full_teams"] >= 1 and st["teams"] < count
    assert teams[0][2] == 1
    assert len({(a, b) for a, b, _ in teams}) == count
    assert np.array_equal(out.cpu().numpy(), ref_out.cpu().numpy())
    assert np.array_equal(np.array(amax), ref_amax.cpu().numpy())


def test_auxiliary_kernel_in_a_region(dev):
    k, n = 10, 5000
    rng = np.random.default_rng(812)
    xs = [torch.from_numpy(rng.standard_normal(n)).to(dev) for _ in range(k)]
    ys = [torch.from_numpy(rng.standard_normal(n)).to(dev) for _ in range(k)]
    outs = [torch.full((n,), float("nan"), dtype=torch.float64, device=dev) for _ in range(k)]
    coef = [(0.75, 0.25), (1 / 3, 2 / 3)] * (k // 2)
    region = hydroagg.Region(max_team=4, n_streams=2, arena_bytes=1 << 14)
    kernel = hydroagg.region_kernel(hydroagg.REGION_AXPBY)
    bpt = (n + 255) // 256

    def task(i):
        def run():
            t = region.enter()
            b, h, _ = region.alloc(t, ctypes.sizeof(hydroagg.hydro_region_axpby_t))
            e = hydroagg.hydro_region_axpby_t(xs[i].data_ptr(), ys[i].data_ptr(),
                                              outs[i].data_ptr(), coef[i][0], coef[i][1], n)
            ctypes.memmove(h, ctypes.byref(e), ctypes.sizeof(e))
            region.upload(t, b)
            base, _ = region.buffer(t, b)
            region.launch(t, kernel, bpt, 256, [ctypes.c_void_p(base), ctypes.c_int32(t.size),
                                                ctypes.c_int32(bpt)])
            region.leave(t)
        return run
    _run_threads([task(i) for i in range(k)])
    st = region.stats()
    region.close()
    assert st["tasks"] == k and st["launches"] == st["teams"]
    for i in range(k):
        want = coef[i][0] * xs[i].cpu().numpy() + coef[i][1] * ys[i].cpu().numpy()
        got = outs[i].cpu().numpy()
        assert np.max(np.abs(got - want)) <= 1e-15 * np.max(np.abs(want)), i


@pytest.mark.parametrize("mode", ["region", "each"])
def test_task_driver_matches_hydro_step(dev, mode):
    count, nf, dt, dx = 512, 11, 0.002, 0.05
    print(f"region driver: {count} tasks, 16 threads, mode {mode}", flush=True)
    U = workloads.random_smooth(count, n=8, nfields=nf, seed=813)
    u_in = torch.from_numpy(U).to(dev)
    ref_out = torch.full((count, nf, 8, 8, 8), float("nan"), dtype=torch.float64, device=dev)
    ref_amax = torch.zeros(count, dtype=torch.float64, device=dev)
    hydroagg.hydro_step(hydroagg.subgrids(u_in, ref_out), dt, dx, ref_amax)
    torch.cuda.synchronize()
    out = torch.full_like(ref_out, float("nan"))
    amax = np.zeros(count)
    region = hydroagg.Region(max_team=64, n_streams=2, arena_bytes=1 << 16) if mode == "region" else None
    secs = hydroagg.region_drive(region, hydroagg.subgrids(u_in, out), dt, dx, 16,
                                 hydroagg.DRIVE_REGION if mode == "region" else hydroagg.DRIVE_EACH,
                                 amax)
    torch.cuda.synchronize()
    if region is not None:
        st = region.stats()
        region.close()
        print(f"  {secs * 1e3:.1f} ms, stats {st}", flush=True)
        assert st["tasks"] == count and st["launches"] == st["teams"] <= count
    assert np.array_equal(out.cpu().numpy(), ref_out.cpu().numpy())
    assert np.array_equal(amax, ref_amax.cpu().numpy())


def test_task_driver_rejects_bad_arguments(dev):
    U = workloads.random_smooth(2, n=8, nfields=11, seed=814)
    u_in = torch.from_numpy(U).to(dev)
    out = torch.empty((2, 11, 8, 8, 8), dtype=torch.float64, device=dev)
    d = hydroagg.subgrids(u_in, out)
    with pytest.raises(hydroagg.HydroError):
        hydroagg.region_drive(None, d, 0.001, 0.05, 4, hydroagg.DRIVE_REGION)   # no region
    with pytest.raises(hydroagg.HydroError):
        hydroagg.region_drive(None, d, 0.001, 0.05, 0, hydroagg.DRIVE_EACH)     # no threads
