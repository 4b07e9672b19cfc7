"""The oracle's branch and positivity counters on the three step workloads.

The method has no floors or positivity fixes (reading R18): it relies on the
limited reconstruction of primitive rho and p keeping both positive at every
cell and face-centre state.  These tests pin that claim on the inputs the
GPU path is measured on -- no non-positive density or pressure at any cell a
stencil reads or at any face state -- and show that every case of the
monotonised-central slope (Colella & Woodward 1984, eq. 1.8) and of the
parabola constraint (eq. 1.10) is taken on each of them, including inside
sub-grids that hold only the 1e-10 atmosphere of the polytrope.
"""
import numpy as np
import pytest

from paper_2210_06438_amd import workloads

BRANCHES = ("slope_zero", "slope_central", "slope_limited",
            "par_flat", "par_left", "par_right", "par_keep")


def _counts(oracle_mod, U, dx, levels=None):
    _, _, c = oracle_mod.step(U, 0.0, dx, levels=levels, counters=True)
    return c


def _assert_counts(c, what):
    assert c["nonpos_cell"] == 0 and c["nonpos_face"] == 0, (what, c)
    for b in BRANCHES:
        assert c[b] > 0, (what, b, c)


def test_brick_counts(oracle_mod):
    c = _counts(oracle_mod, workloads.brick(seed=1), 1 / 64)
    _assert_counts(c, "brick")
    # every reconstructed value falls in exactly one slope case and one
    # parabola case: 3 directions x n^2 lines x F fields per sub-grid, the
    # slope at 12 cells and the parabola at 10 cells per line
    lines = 8 * 3 * 64 * 6
    assert c["slope_zero"] + c["slope_central"] + c["slope_limited"] == lines * 12
    assert c["par_flat"] + c["par_left"] + c["par_right"] + c["par_keep"] == lines * 10


def test_random_smooth_counts(oracle_mod):
    _assert_counts(_counts(oracle_mod, workloads.random_smooth(64, n=8, nfields=11, seed=2), 1 / 64),
                   "random smooth, first 64 of the 4096 sub-grids")


@pytest.mark.slow
def test_polytrope_3000_counts(oracle_mod):
    groups = workloads.polytrope(count=3000, seed=3)
    total = {}
    atm_total = {}
    for N, levels, U, _ in groups:
        c = _counts(oracle_mod, U, 0.5, levels)
        _assert_counts(c, f"polytrope n={N}")
        for k, v in c.items():
            total[k] = total.get(k, 0) + v
        atm = np.all(U[:, 0] <= workloads.ATMOSPHERE, axis=(1, 2, 3))
        assert atm.any()
        ca = _counts(oracle_mod, U[atm], 0.5, levels[atm])
        _assert_counts(ca, f"polytrope n={N}, atmosphere-only sub-grids")
        for k, v in ca.items():
            atm_total[k] = atm_total.get(k, 0) + v
    print("polytrope counters", total, "atmosphere only", atm_total)
