"""Seeded synthetic sub-grid inputs shared by the tests, the smoke check and
the benchmark.

This module only *draws* inputs: it builds conserved states from a recipe of
primitive fields (the ideal-gas energy E = p/(gamma-1) + rho|v|^2/2 is part of
the recipe) and fills ghost layers by periodic wrap.  It contains none of the
step's arithmetic (no reconstruction, flux or update) and imports neither the
HIP path nor the oracle.

Layout of every array returned: float64 [count, F, M, M, M], M = N + 6, SoA
with x fastest.  Fields: 0 rho, 1 sx, 2 sy, 3 sz, 4 egas, 5 tau, 6..10 the
partial densities rho_k of five species (F = 11 only).

Workloads (the paper's own benchmark, a Sedov blast on 512 sub-grids of 8^3,
Section VI-A and Table II, has no released inputs; these seeded states stand
in for it, with the same sub-grid shape and FP64 fields):
  * ``brick``       8 sub-grids of 8^3, F=6, a 2x2x2 periodic brick (16^3).
  * ``random_smooth`` independent sub-grids, 10% iid perturbations.
  * ``polytrope``   mixed edges {8, 12, 16}, density of an n=1.5 polytrope
                    sampled at random octree positions, 1e-10 floor.
Every sub-grid is drawn from its own generator ``PCG64(SeedSequence([seed,
s]))`` so any one can be regenerated alone; within a sub-grid the draw order
is cell (z, y, x) then variable.
"""
from __future__ import annotations

import numpy as np

GAMMA = 5.0 / 3.0
GHOST = 3
ATMOSPHERE = 1e-10


def _rng(seed: int, s: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(s)])))


def conserved_from_primitive(rho, vx, vy, vz, p, species_frac=None):
    """Initial-condition recipe: primitive fields -> stored fields.
    tau = (p/(gamma-1))^(1/gamma); rho_k = rho * X_k.  Arrays broadcast."""
    e_int = p / (GAMMA - 1.0)
    fields = [rho, rho * vx, rho * vy, rho * vz,
              e_int + 0.5 * rho * (vx * vx + vy * vy + vz * vz),
              e_int ** (1.0 / GAMMA)]
    if species_frac is not None:
        for k in range(species_frac.shape[-1]):
            fields.append(rho * species_frac[..., k])
    return np.stack(fields, axis=0)


def _smooth_block(rng, shape, nfields):
    """rho, p = 1 + 0.1 U(-1,1); v_d = U(-0.1, 0.1); species ~ Dirichlet(1)."""
    u = rng.uniform(-1.0, 1.0, size=shape + (5,))
    rho = 1.0 + 0.1 * u[..., 0]
    p = 1.0 + 0.1 * u[..., 1]
    vx, vy, vz = 0.1 * u[..., 2], 0.1 * u[..., 3], 0.1 * u[..., 4]
    X = rng.dirichlet(np.ones(5), size=shape) if nfields == 11 else None
    return conserved_from_primitive(rho, vx, vy, vz, p, X)


def random_smooth(count: int, n: int = 8, nfields: int = 11, seed: int = 2,
                  start: int = 0) -> np.ndarray:
    """Independent sub-grids; each full (n+6)^3 block, ghosts included, drawn
    iid per cell.  ``start`` offsets the sub-grid index (to regenerate a
    slice of a larger batch)."""
    if nfields not in (6, 11):
        raise ValueError("nfields must be 6 or 11")
    M = n + 2 * GHOST
    out = np.empty((count, nfields, M, M, M), dtype=np.float64)
    for i in range(count):
        out[i] = _smooth_block(_rng(seed, start + i), (M, M, M), nfields)
    return out


def periodic_tiles(U: np.ndarray, per_axis: int, n: int) -> np.ndarray:
    """Cut a periodic global field U[F, Z, Y, X] (Z=Y=X=per_axis*n) into
    per_axis^3 sub-grids with 3-deep ghosts filled by periodic wrap (edges and
    corners included).  Sub-grid order: (bz, by, bx), bx fastest."""
    nf = U.shape[0]
    M = n + 2 * GHOST
    L = per_axis * n
    idx = lambda b: (np.arange(-GHOST, n + GHOST) + b * n) % L
    out = np.empty((per_axis ** 3, nf, M, M, M), dtype=np.float64)
    s = 0
    for bz in range(per_axis):
        for by in range(per_axis):
            for bx in range(per_axis):
                out[s] = U[:, idx(bz)][:, :, idx(by)][:, :, :, idx(bx)]
                s += 1
    return out


def brick(seed: int = 1, n: int = 8, per_axis: int = 2, nfields: int = 6) -> np.ndarray:
    """A per_axis^3 brick of n^3 sub-grids tiling a periodic domain; the global
    field is drawn once with the smooth recipe (draw order: cell (z, y, x),
    then variable)."""
    L = per_axis * n
    rng = np.random.Generator(np.random.PCG64(seed))
    U = _smooth_block(rng, (L, L, L), nfields)
    return periodic_tiles(U, per_axis, n)


# --------------------------------------------------------------------------
# n = 1.5 polytrope (Lane-Emden), for the uneven-size workload
# --------------------------------------------------------------------------
_LE_TABLE = None


def lane_emden_table(n_index: float = 1.5, h: float = 1e-4):
    """theta(xi) of the Lane-Emden equation theta'' + 2 theta'/xi + theta^n = 0,
    theta(0)=1, theta'(0)=0, by classical RK4 up to the first zero xi_1.
    Returns (xi[], theta[], xi_1)."""
    global _LE_TABLE
    if _LE_TABLE is not None and _LE_TABLE[3] == (n_index, h):
        return _LE_TABLE[:3]

    def rhs(xi, th, dth):
        return dth, -(max(th, 0.0) ** n_index) - 2.0 * dth / xi

    xi = h
    th = 1.0 - xi * xi / 6.0 + n_index * xi ** 4 / 120.0   # series start
    dth = -xi / 3.0 + n_index * xi ** 3 / 30.0
    xs, ts = [0.0, xi], [1.0, th]
    while th > 0.0:
        k1 = rhs(xi, th, dth)
        k2 = rhs(xi + h / 2, th + h / 2 * k1[0], dth + h / 2 * k1[1])
        k3 = rhs(xi + h / 2, th + h / 2 * k2[0], dth + h / 2 * k2[1])
        k4 = rhs(xi + h, th + h * k3[0], dth + h * k3[1])
        th_new = th + h / 6 * (k1[0] + 2 * k2[0] + 2 * k3[0] + k4[0])
        dth_new = dth + h / 6 * (k1[1] + 2 * k2[1] + 2 * k3[1] + k4[1])
        if th_new <= 0.0:
            xi1 = xi + h * th / (th - th_new)           # linear root in the last step
            xs.append(xi1)
            ts.append(0.0)
            xi, th = xi1, 0.0
            break
        xi, th, dth = xi + h, th_new, dth_new
        xs.append(xi)
        ts.append(th)
    _LE_TABLE = (np.array(xs), np.array(ts), xs[-1], (n_index, h))
    return _LE_TABLE[:3]


def polytrope(count: int = 3000, seed: int = 3, nfields: int = 11,
              edges=(8, 12, 16), probs=(0.7, 0.2, 0.1), dx: float = 0.5,
              levels=(2, 3, 4, 5), radius: float = 1.0, half_width: float = 2.0):
    """Sub-grids of an n=1.5 polytrope (radius 1, centred in [-2, 2]^3).

    Per sub-grid s (own generator): edge N_s from ``edges`` with ``probs``;
    octree level L_s uniform in ``levels``; cell width h_s = dx * 2^-L_s (the
    descriptor's level semantics); node index uniform so the sub-grid lies in
    the domain.  Cells (ghosts included) sample at their centres:
    rho = max(theta(xi_1 r/R)^1.5, 1e-10), p = rho^(5/3) (K = 1),
    v_d = 0.1 c_s U(-1,1) with c_s = sqrt(gamma p / rho), species ~ Dirichlet(1).

    Returns a list of (edge, levels[int64], U[count_e, F, M, M, M], index[])
    groups, one per edge present, where index[] is each sub-grid's position s
    in the drawn sequence.
    """
    xs, ts, xi1 = lane_emden_table()
    groups = {}
    for s in range(count):
        rng = _rng(seed, s)
        N = int(edges[rng.choice(len(edges), p=probs)])
        L = int(levels[rng.integers(len(levels))])
        h = dx * 2.0 ** (-L)
        nodes = max(int(np.floor(2 * half_width / (N * h))), 1)
        node = rng.integers(0, nodes, size=3)
        M = N + 2 * GHOST
        c = -half_width + (node[:, None] * N + np.arange(-GHOST, N + GHOST)[None, :] + 0.5) * h
        zc, yc, xc = np.meshgrid(c[2], c[1], c[0], indexing="ij")
        r = np.sqrt(xc * xc + yc * yc + zc * zc)
        th = np.interp(xi1 * r / radius, xs, ts, right=0.0)
        rho = np.maximum(np.clip(th, 0.0, None) ** 1.5, ATMOSPHERE)
        p = rho ** GAMMA
        cs = np.sqrt(GAMMA * p / rho)
        u = rng.uniform(-1.0, 1.0, size=(M, M, M, 3))
        vx, vy, vz = (0.1 * cs * u[..., k] for k in range(3))
        X = rng.dirichlet(np.ones(5), size=(M, M, M)) if nfields == 11 else None
        U = conserved_from_primitive(rho, vx, vy, vz, p, X)
        groups.setdefault(N, []).append((s, L, U))
    out = []
    for N in sorted(groups):
        g = groups[N]
        out.append((N, np.array([x[1] for x in g], dtype=np.int64),
                    np.stack([x[2] for x in g]), np.array([x[0] for x in g], dtype=np.int64)))
    return out


def cells(n: int) -> int:
    return n ** 3


def ghost_cells(n: int) -> int:
    """(n+6)^3 - n^3 stored ghost cells per sub-grid."""
    return (n + 2 * GHOST) ** 3 - n ** 3
