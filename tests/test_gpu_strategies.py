"""The paper's strategies on the GPU (Section V): strategy 2 (one launch per
sub-grid over a pool of streams) and strategy 3 / the 2+3 combination (the
aggregator with up to 128 streams, tasks arriving as a burst) give every
sub-grid bitwise the result and amax of the aggregated step."""
import numpy as np
import pytest

from paper_2210_06438_amd import hydroagg, workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PARTS = [(8, 11, 23, 701), (12, 6, 5, 702), (16, 11, 3, 703)]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _batch(dev, nan=True):
    ins, outs, descs = [], [], []
    for n, nf, count, seed in PARTS:
        u = torch.from_numpy(workloads.random_smooth(count, n=n, nfields=nf, seed=seed)).to(dev)
        o = torch.full((count, nf, n, n, n), float("nan"), dtype=torch.float64, device=dev)
        ins.append(u)
        outs.append(o)
        descs.append(hydroagg.subgrids(u, o, levels=[i % 2 for i in range(count)]))
    d = hydroagg.concat(*descs)
    return ins, outs, d, torch.full((d[1],), float("nan"), dtype=torch.float64, device=dev)


def _reference(dev, dt, dx):
    _, outs, d, amax = _batch(dev)
    hydroagg.hydro_step(d, dt, dx, amax)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs], amax.cpu().numpy()


@pytest.mark.parametrize("k", [1, 3, 128])
def test_strategy2_streams_match_the_aggregated_step(dev, k):
    dt, dx = 0.002, 0.05
    print(f"strategy 2: {k} streams", flush=True)
    ref, ref_amax = _reference(dev, dt, dx)
    _, outs, d, amax = _batch(dev)
    hydroagg.hydro_step_streams(d, dt, dx, amax, n_streams=k)
    # ordered on the caller's stream: the copies below wait for every pool stream
    got = [o.cpu().numpy() for o in outs]
    assert np.array_equal(amax.cpu().numpy(), ref_amax)
    for g, r in zip(got, ref):
        assert np.array_equal(g, r)


@pytest.mark.parametrize("width,streams", [(1, 1), (8, 16), (16, 128)])
def test_bulk_submit_over_many_streams_matches_the_aggregated_step(dev, width, streams):
    dt, dx = 0.002, 0.05
    print(f"aggregator: width {width}, {streams} streams, burst submit", flush=True)
    ref, ref_amax = _reference(dev, dt, dx)
    _, outs, d, _ = _batch(dev)
    agg = hydroagg.Aggregator(width, timeout_us=-1.0, n_streams=streams, flush_when_idle=True)
    tickets = agg.submit_many(d, dt, dx, tickets=True)
    amax = np.array([agg.wait(int(t)) for t in tickets])
    st = agg.stats()
    agg.close()
    assert st["submitted"] == d[1] and st["launched"] == d[1]
    assert np.array_equal(amax, ref_amax)
    for o, r in zip(outs, ref):
        assert np.array_equal(o.cpu().numpy(), r)


def test_fire_and_forget_burst_then_drain(dev):
    dt, dx = 0.002, 0.05
    ref, _ = _reference(dev, dt, dx)
    _, outs, d, _ = _batch(dev)
    agg = hydroagg.Aggregator(4, timeout_us=-1.0, n_streams=8, flush_when_idle=True)
    for _ in range(3):   # the same burst three times, as the iterations of a time-step
        assert agg.submit_many(d, dt, dx) is None
        agg.drain()
    st = agg.stats()
    agg.close()
    assert st["launched"] == 3 * d[1] and st["held"] == 0
    for o, r in zip(outs, ref):
        assert np.array_equal(o.cpu().numpy(), r)
