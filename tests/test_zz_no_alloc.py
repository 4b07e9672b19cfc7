"""hydro_step_static, the step that allocates nothing (its descriptor table is
a static device array), against hydro_step on the same inputs: bitwise equal
outputs and amax, for two calls in a row on one stream (the second with a
smaller batch, issued before the first has finished), and for a batch of
the table's full size."""
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


def _batch(dev, parts):
    """parts: list of (n, nfields, count, seed); device inputs, outputs
    (NaN), descriptors and an amax array."""
    ins, outs, descs = [], [], []
    for n, nf, count, seed in parts:
        u = torch.from_numpy(workloads.random_smooth(count, n=n, nfields=nf, seed=seed)).to(dev)
        o = torch.full_like(u, float("nan"))
        ins.append(u)
        outs.append(o)
        descs.append(hydroagg.subgrids(u, o, levels=[(i % 3) for i in range(count)]))
    d = hydroagg.concat(*descs)
    amax = torch.full((d[1],), float("nan"), dtype=torch.float64, device=dev)
    return ins, outs, d, amax


def _reference(dev, parts, dt, dx):
    ins, outs, d, amax = _batch(dev, parts)
    hydroagg.hydro_step(d, dt, dx, amax)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs], amax.cpu().numpy()


def _same(tag, got_outs, got_amax, ref_outs, ref_amax):
    for j, (g, r) in enumerate(zip(got_outs, ref_outs)):
        g = g.cpu().numpy()
        assert np.array_equal(g, r, equal_nan=True), f"{tag}: part {j} differs from hydro_step"
    assert np.array_equal(got_amax.cpu().numpy(), ref_amax), f"{tag}: amax differs from hydro_step"


# first call: a multi-class batch of 11 fields (one launch from the table);
# second call, smaller: two classes of two field counts, one of them beyond the
# argument-carried size (per-class launches, table and arguments)
FIRST = [(8, 11, 300, 901), (12, 11, 40, 902), (16, 11, 20, 903)]
SECOND = [(8, 6, 30, 904), (16, 11, 5, 905)]


def test_two_static_calls_in_a_row_match_hydro_step(dev):
    dt, dx = 0.002, 0.05
    print("no-alloc: references through hydro_step", flush=True)
    ref1 = _reference(dev, FIRST, dt, dx)
    ref2 = _reference(dev, SECOND, dt, dx)
    ins1, outs1, d1, amax1 = _batch(dev, FIRST)
    ins2, outs2, d2, amax2 = _batch(dev, SECOND)
    torch.cuda.synchronize()
    print(f"no-alloc: hydro_step_static of {d1[1]} then {d2[1]} sub-grids, no wait between",
          flush=True)
    hydroagg.hydro_step_static(d1, dt, dx, amax1)
    hydroagg.hydro_step_static(d2, dt, dx, amax2)
    torch.cuda.synchronize()
    _same("first call", outs1, amax1, *ref1)
    _same("second call", outs2, amax2, *ref2)
    # and once more, the larger batch after the smaller one
    for o in outs1:
        o.fill_(float("nan"))
    amax1.fill_(float("nan"))
    hydroagg.hydro_step_static(d1, dt, dx, amax1)
    torch.cuda.synchronize()
    _same("third call", outs1, amax1, *ref1)


def test_static_call_at_the_table_size_matches_hydro_step(dev):
    dt, dx = 0.003, 0.05
    parts = [(8, 6, hydroagg.STATIC_MAX, 906)]
    print(f"no-alloc: {hydroagg.STATIC_MAX} sub-grids (the table size)", flush=True)
    ref = _reference(dev, parts, dt, dx)
    ins, outs, d, amax = _batch(dev, parts)
    hydroagg.hydro_step_static(d, dt, dx, amax)
    torch.cuda.synchronize()
    _same("full table", outs, amax, *ref)
