"""CPU oracle of the multi-stage time-step on a brick of sub-grids -- TEST
INFRASTRUCTURE ONLY (same rules as the rest of ``oracle/``: only tests, the
smoke check and the CPU-baseline leg of the benchmark load it; it shares no
code with the HIP path).

A brick is nb = (nbx, nby, nbz) sub-grids of edge n tiling a rectangular
domain of n*nb cells per axis, sub-grid s = (bz*nby + by)*nbx + bx, each
stored with 3 ghost layers as [F, M, M, M] (M = n + 6), the layout the hydro
step reads (Section V-A of the paper: sub-grids with ghost layers filled
from their neighbours).  The paper's time-step is three solver iterations
(Section VI-A); read here as the three-stage SSP Runge-Kutta method of Shu
and Osher (J. Comput. Phys. 77, 1988, eq. 2.18):

    U1 = E(U0),   U2 = 3/4 U0 + 1/4 E(U1),   U3 = 1/3 U0 + 2/3 E(U2)

with E(V) = V + dt L(V) one forward-Euler hydro stage (``oracle.step``) and
every stage result's ghost layers refilled before the next stage reads them.

Pins: ``tests/test_oracle_brick.py`` (periodic fill against the input
generator's independent periodic tiling, outflow fill against numpy edge
padding, the stage combination against the third-order Taylor polynomial of
a linear problem, fixed point and conservation with the hydro stage).
"""
from __future__ import annotations

import numpy as np

GHOST = 3
PERIODIC = 0
OUTFLOW = 1


def _domain_index(g: int, L: int, bc: int) -> int:
    """Domain cell that cell coordinate g stands for: periodic wrap, or the
    outermost cell beyond an outflow (zero-gradient) boundary."""
    if bc == PERIODIC:
        return g % L
    return min(max(g, 0), L - 1)


def ghost_fill(U: np.ndarray, nb, bc) -> np.ndarray:
    """Copy of the brick U [count, F, M, M, M] with every ghost cell (faces,
    edges, corners) set to the domain cell it stands for, per axis
    independently.  Interior cells are returned unchanged."""
    U = np.asarray(U, dtype=np.float64)
    count, nf, M = U.shape[0], U.shape[1], U.shape[2]
    n = M - 2 * GHOST
    nbx, nby, nbz = (int(v) for v in nb)
    if count != nbx * nby * nbz:
        raise ValueError("count does not match nb")
    L = (n * nbx, n * nby, n * nbz)
    # per axis and per sub-grid position along it: for every stored
    # coordinate, the (sub-grid position, stored coordinate) of its source
    maps = []
    for d, nbd in enumerate((nbx, nby, nbz)):
        src_b = np.empty((nbd, M), dtype=np.int64)
        src_c = np.empty((nbd, M), dtype=np.int64)
        for b in range(nbd):
            for c in range(M):
                g = _domain_index(b * n + c - GHOST, L[d], int(bc[d]))
                src_b[b, c] = g // n
                src_c[b, c] = g % n + GHOST
        maps.append((src_b, src_c))
    out = U.copy()
    interior = np.zeros((M, M, M), dtype=bool)
    interior[GHOST:GHOST + n, GHOST:GHOST + n, GHOST:GHOST + n] = True
    ghost = ~interior
    z, y, x = np.nonzero(ghost)
    for bz in range(nbz):
        for by in range(nby):
            for bx in range(nbx):
                s = (bz * nby + by) * nbx + bx
                sb = (maps[2][0][bz, z] * nby + maps[1][0][by, y]) * nbx + maps[0][0][bx, x]
                out[s][:, z, y, x] = U[sb, :, maps[2][1][bz, z], maps[1][1][by, y],
                                       maps[0][1][bx, x]].T
    return out


def rk3_stages(stage, U0: np.ndarray, nb, bc):
    """The three SSP-RK3 stages from the filled state U0.  ``stage(V)`` is
    the forward-Euler stage E(V) (interior updated; ghosts are refilled here
    before the next stage).  Returns (U1, U2, U3), each with ghosts filled."""
    U0 = np.asarray(U0, dtype=np.float64)
    U1 = ghost_fill(stage(U0), nb, bc)
    U2 = ghost_fill(0.75 * U0 + 0.25 * stage(U1), nb, bc)
    U3 = ghost_fill((1.0 / 3.0) * U0 + (2.0 / 3.0) * stage(U2), nb, bc)
    return U1, U2, U3
