"""Pins of the brick oracle (ghost fill and the SSP-RK3 composition of the
hydro stage) against independent constructions and closed forms."""
import math

import numpy as np
import pytest

from oracle import brick as ob
from paper_2210_06438_amd import workloads


def _tiles_from_global(G, nb, n, modes):
    """Cut the global interior field G [F, Lz, Ly, Lx] into sub-grids with
    3-deep ghosts by numpy padding (modes per axis x, y, z: 'wrap' or
    'edge'); an independent construction of the filled brick."""
    P = G
    for axis, mode in zip((3, 2, 1), modes):
        pad = [(0, 0)] * 4
        pad[axis] = (3, 3)
        P = np.pad(P, pad, mode=mode)
    M = n + 6
    out = []
    for bz in range(nb[2]):
        for by in range(nb[1]):
            for bx in range(nb[0]):
                out.append(P[:, bz * n:bz * n + M, by * n:by * n + M, bx * n:bx * n + M])
    return np.stack(out)


def _random_brick(rng, nb, n, nf):
    """A brick whose interiors are random and whose ghosts hold NaN."""
    M = n + 6
    U = np.full((nb[0] * nb[1] * nb[2], nf, M, M, M), np.nan)
    U[:, :, 3:3 + n, 3:3 + n, 3:3 + n] = rng.uniform(0.5, 1.5, size=(len(U), nf, n, n, n))
    return U


def _global(U, nb, n):
    nf = U.shape[1]
    G = np.empty((nf, nb[2] * n, nb[1] * n, nb[0] * n))
    for bz in range(nb[2]):
        for by in range(nb[1]):
            for bx in range(nb[0]):
                s = (bz * nb[1] + by) * nb[0] + bx
                G[:, bz * n:(bz + 1) * n, by * n:(by + 1) * n, bx * n:(bx + 1) * n] = \
                    U[s, :, 3:3 + n, 3:3 + n, 3:3 + n]
    return G


def test_periodic_fill_matches_the_input_generators_tiling():
    rng = np.random.default_rng(1)
    for nb, n in (((2, 2, 2), 8), ((3, 1, 2), 12), ((1, 1, 1), 8)):
        U = _random_brick(rng, nb, n, 6)
        got = ob.ghost_fill(U, nb, (0, 0, 0))
        G = _global(U, nb, n)
        if nb[0] == nb[1] == nb[2]:
            assert np.array_equal(got, workloads.periodic_tiles(G, nb[0], n))
        assert np.array_equal(got, _tiles_from_global(G, nb, n, ("wrap",) * 3))


@pytest.mark.parametrize("bc", [(1, 0, 0), (1, 1, 1), (0, 1, 0), (0, 0, 1)])
def test_outflow_and_mixed_fill_match_numpy_padding(bc):
    rng = np.random.default_rng(2)
    nb, n = (3, 2, 1), 8
    U = _random_brick(rng, nb, n, 11)
    got = ob.ghost_fill(U, nb, bc)
    modes = tuple("edge" if b == ob.OUTFLOW else "wrap" for b in bc)
    assert np.array_equal(got, _tiles_from_global(_global(U, nb, n), nb, n, modes))
    # interiors untouched, idempotent
    assert np.array_equal(got[:, :, 3:11, 3:11, 3:11], U[:, :, 3:11, 3:11, 3:11])
    assert np.array_equal(ob.ghost_fill(got, nb, bc), got)


def test_stage_combination_is_the_third_order_taylor_polynomial():
    """With E(V) = (1 + z) V, a linear stage, the three stages give
    U3 = (1 + z + z^2/2 + z^3/6) U0: the SSP-RK3 stability polynomial."""
    nb, n = (2, 1, 1), 8
    rng = np.random.default_rng(3)
    U0 = ob.ghost_fill(_random_brick(rng, nb, n, 6), nb, (0, 0, 0))
    for z in (-0.3, 0.1, 0.7):
        U1, U2, U3 = ob.rk3_stages(lambda V: (1.0 + z) * V, U0, nb, (0, 0, 0))
        poly = 1 + z + z * z / 2 + z ** 3 / 6
        assert np.allclose(U3, poly * U0, rtol=1e-15, atol=0)
        assert np.allclose(U2, (1 + z / 2 + z * z / 4) * U0, rtol=1e-15, atol=0)
        assert np.allclose(U1, (1 + z) * U0, rtol=1e-15, atol=0)


def test_uniform_state_is_a_fixed_point_of_the_time_step(oracle_mod):
    nb, n, M = (2, 2, 1), 8, 14
    W = [1.3, 0.2, -0.4, 0.7, 2.1, 0.3]
    e = W[4] / (5 / 3 - 1) + 0.5 * W[0] * (W[1] ** 2 + W[2] ** 2 + W[3] ** 2)
    Uc = np.array([W[0], W[0] * W[1], W[0] * W[2], W[0] * W[3], e, W[5]])
    U0 = np.broadcast_to(Uc[None, :, None, None, None], (4, 6, M, M, M)).copy()
    stages = ob.rk3_stages(lambda V: oracle_mod.step(V, 0.01, 0.02)[0], U0, nb, (0, 1, 0))
    for S in stages:
        assert np.allclose(S, U0, rtol=2e-16, atol=0)


def test_time_step_conserves_totals_on_a_periodic_brick(oracle_mod):
    U0 = workloads.brick(seed=6)
    nb = (2, 2, 2)
    dx = 1 / 64
    _, a = oracle_mod.step(U0, 0.0, dx)
    dt = 0.4 * dx / a.max()
    _, _, U3 = ob.rk3_stages(lambda V: oracle_mod.step(V, dt, dx)[0], U0, nb, (0, 0, 0))
    for f in range(U0.shape[1]):
        before = math.fsum(U0[:, f, 3:11, 3:11, 3:11].ravel())
        after = math.fsum(U3[:, f, 3:11, 3:11, 3:11].ravel())
        scale = math.fsum(np.abs(U0[:, f, 3:11, 3:11, 3:11]).ravel())
        assert abs(after - before) <= 1e-13 * scale
    # the filled state the generator made is the filled state the oracle makes
    assert np.array_equal(ob.ghost_fill(U0, nb, (0, 0, 0)), U0)
