"""The scheme converges: Sod's shock tube on strips of 8^3 sub-grids, three
oracle stages per step composed into SSP-RK3 on the host (the paper's time
step is three solver iterations, Section VI-A), against the exact Riemann
solution.  Also pins the exact solver, the Lane-Emden table used to draw the
polytrope workload, and the sub-grid sizing of the paper's Table II."""
import math
import os

import numpy as np
import pytest

from paper_2210_06438_amd import workloads
from tests.ref import euler, riemann

HERE = os.path.dirname(os.path.abspath(__file__))
G = 5.0 / 3.0
LEFT = (1.0, 0.0, 1.0)
RIGHT = (0.125, 0.0, 0.1)


def _golden(name):
    rows = []
    with open(os.path.join(HERE, "golden", name)) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([float(x) for x in line.split()])
    return np.array(rows)


def test_exact_solver_matches_published_sod_star_state():
    ps, us, rl, rr = _golden("sod_star_gamma14.txt")[0]
    p, u, rL, rR = riemann.star_state(LEFT, RIGHT, 1.4)
    assert abs(p - ps) < 5e-6 and abs(u - us) < 5e-6
    assert abs(rL - rl) < 5e-6 and abs(rR - rr) < 5e-6


def test_exact_solver_solution_is_consistent():
    """Sampled solution: far field equals the data; the contact carries p*, u*."""
    for g in (1.4, G):
        ps, us, rL, rR = riemann.star_state(LEFT, RIGHT, g)
        rho, u, p = riemann.sample(LEFT, RIGHT, g, np.array([-5.0, us - 1e-9, us + 1e-9, 5.0]))
        assert rho[0] == 1.0 and rho[-1] == 0.125
        assert p[1] == pytest.approx(ps) and p[2] == pytest.approx(ps)
        assert u[1] == pytest.approx(us) and rho[1] == pytest.approx(rL) and rho[2] == pytest.approx(rR)


def test_lane_emden_first_zero():
    """n = 1.5 polytrope: xi_1 = 3.65375 (S. Chandrasekhar, An Introduction to
    the Study of Stellar Structure, 1939, ch. IV)."""
    _, _, xi1 = workloads.lane_emden_table()
    assert abs(xi1 - 3.65375) < 2e-5


def test_table2_sizing():
    for edge, total, leaves, ghosts, calls, transfers, items in _golden("table2_sizes.txt"):
        edge = int(edge)
        assert workloads.ghost_cells(edge) == ghosts
        assert leaves * workloads.cells(edge) == total
        assert 5 * 3 * leaves == calls            # 5 kernels x 3 iterations per step
        assert 2 * calls == transfers
        assert (edge + 2) ** 3 == items          # interior plus the innermost ghost layer


def _fill_strip(Uint, nsub, n=8):
    """Interior strip [F, n, n, n*nsub] -> nsub sub-grids with ghosts:
    zero-gradient (outflow) at the x ends, periodic in y and z."""
    P = np.pad(Uint, ((0, 0), (3, 3), (3, 3), (0, 0)), mode="wrap")
    P = np.pad(P, ((0, 0), (0, 0), (0, 0), (3, 3)), mode="edge")
    return np.stack([P[..., n * s:n * s + n + 6] for s in range(nsub)])


def _gather(Us, nsub, n=8):
    return np.concatenate([Us[s][:, 3:3 + n, 3:3 + n, 3:3 + n] for s in range(nsub)], axis=-1)


def _sod_l1(oracle_mod, nsub, t_end=0.2, cfl=0.4, n=8):
    cells = n * nsub
    dx = 1.0 / cells
    x = (np.arange(cells) + 0.5) * dx
    W = np.zeros((6, n, n, cells))
    left = x < 0.5
    W[0] = np.where(left, LEFT[0], RIGHT[0])
    W[4] = np.where(left, LEFT[2], RIGHT[2])
    W[5] = 1.0
    U = euler.cons(W)
    t = 0.0

    def stage(Uint, dt):
        out, amax = oracle_mod.step(_fill_strip(Uint, nsub), dt=dt, dx=dx)
        return _gather(out, nsub), amax

    while t < t_end - 1e-14:
        _, amax = stage(U, 0.0)
        dt = min(cfl * dx / amax.max(), t_end - t)
        U1, _ = stage(U, dt)
        U2, _ = stage(U1, dt)
        U2 = 0.75 * U + 0.25 * U2
        U3, _ = stage(U2, dt)
        U = U / 3.0 + 2.0 / 3.0 * U3
        t += dt
    # every y-z line is identical
    assert np.max(np.abs(U[0] - U[0, :1, :1, :])) < 1e-12
    rho_ex, _, _ = riemann.sample(LEFT, RIGHT, G, (x - 0.5) / t_end)
    return np.mean(np.abs(U[0, 0, 0] - rho_ex))


@pytest.mark.slow
def test_sod_converges_to_the_exact_solution(oracle_mod):
    head, shock = riemann.wave_positions(LEFT, RIGHT, G)
    assert 0.0 < 0.5 + head * 0.2 and 0.5 + shock * 0.2 < 1.0     # waves stay inside
    errs = [_sod_l1(oracle_mod, nsub) for nsub in (4, 8, 16)]
    assert errs[0] / errs[1] >= 1.6 and errs[1] / errs[2] >= 1.6, errs
    assert errs[2] < 5e-3, errs
