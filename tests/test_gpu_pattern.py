"""The access-pattern reference kernel (hydro_plan_pattern_floor) touches
exactly the cells the step does: on inputs of magnitude ~1 the value it
writes is the input interior cell itself (the added multiple of the ghost
sum, 1e-300 times it, is far below half an ulp), so its output must equal
the input interior bitwise, in both output layouts, with the stored
layout's ghost cells left untouched."""
import numpy as np
import pytest

from paper_2210_06438_amd import hydroagg, workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nf", [6, 11])
@pytest.mark.parametrize("same_lds", [True, False])
def test_pattern_kernel_copies_the_interior(nf, same_lds):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    count, n = 37, 8
    print(f"pattern: nf={nf} same_lds={same_lds}", flush=True)
    U = workloads.random_smooth(count, n=n, nfields=nf, seed=77)
    u_in = torch.from_numpy(U).to(dev)
    compact = torch.full((count, nf, n, n, n), float("nan"), dtype=torch.float64, device=dev)
    stored = torch.full_like(u_in, float("nan"))
    inner = U[..., 3:11, 3:11, 3:11]
    for out in (compact, stored):
        plan = hydroagg.Plan(hydroagg.subgrids(u_in, out))
        plan.pattern_floor(same_lds)
        torch.cuda.synchronize()
        plan.close()
    assert np.array_equal(compact.cpu().numpy(), inner)
    got = stored.cpu().numpy()
    assert np.array_equal(got[..., 3:11, 3:11, 3:11], inner)
    got[..., 3:11, 3:11, 3:11] = np.nan
    assert np.all(np.isnan(got))


def test_pattern_kernel_rejects_other_shapes():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    U = workloads.random_smooth(2, n=12, nfields=6, seed=78)
    u_in = torch.from_numpy(U).to(dev)
    plan = hydroagg.Plan(hydroagg.subgrids(u_in, u_in.clone()))
    with pytest.raises(hydroagg.HydroError):
        plan.pattern_floor(True)
    plan.close()
