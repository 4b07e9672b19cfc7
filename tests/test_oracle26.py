"""Pins for the 26-point form of the oracle (oracle.step26: values at the
26 points of each cell's surface, central-upwind fluxes at the 9 points of
every face, Simpson's rule over each face), each against something the
mathematics fixes:

  uniform state          -> a fixed point, bitwise
  linear primitives      -> every one of the 26 point values is the exact
                            value of the linear field at that point
  linear primitives      -> the mass and momentum updates are differences of
                            the EXACT face integrals of the physical flux
                            (3x3 Gauss-Legendre over each face with the
                            textbook flux of tests/ref/euler.py; Simpson's
                            rule is exact for these polynomials, which are
                            at most cubic across a face)
  data varying along x   -> equal to the face-centre form to rounding (all
                            9 points of an x face see the same states, the
                            transverse differences vanish)
  periodic brick         -> conserved totals change only by rounding
  mirror / permutation   -> outputs transform the same way
"""
import math

import numpy as np
import pytest

from paper_2210_06438_amd import workloads
from tests.ref import euler
from tests.test_oracle_pins import (_mirror_x, _swap_xy, _swap_xz, block_from_primitive,
                                    fsum_fields, interior, normwise)

DIRS = [(ex, ey, ez) for ez in (-1, 0, 1) for ey in (-1, 0, 1) for ex in (-1, 0, 1)
        if (ex, ey, ez) != (0, 0, 0)]


def _linear_block(n=8, nf=11, seed=21, scale=0.01):
    """Primitive fields linear in the stored cell index (x, y, z)."""
    M = n + 6
    rng = np.random.default_rng(seed)
    base = np.array([1.0, 0.3, -0.2, 0.1, 2.0, 0.5, 0.1, 0.2, 0.3, 0.25, 0.15])[:nf]
    grad = rng.uniform(-1.0, 1.0, size=(nf, 3)) * scale * np.abs(base)[:, None]
    g = np.arange(M, dtype=np.float64)
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    W = base[:, None, None, None] + grad[:, 0, None, None, None] * X + \
        grad[:, 1, None, None, None] * Y + grad[:, 2, None, None, None] * Z

    def prim_at(x, y, z):
        return base + grad[:, 0] * x + grad[:, 1] * y + grad[:, 2] * z
    return W, prim_at


def test_uniform_state_is_a_fixed_point(oracle_mod):
    U = workloads.random_smooth(1, n=8, nfields=11, seed=31)
    U[:] = U[:, :, :1, :1, :1]
    out, amax = oracle_mod.step26(U, dt=0.01, dx=0.1)
    assert np.array_equal(out, U)
    _, amax6 = oracle_mod.step(U, dt=0.01, dx=0.1)
    assert amax[0] == amax6[0]


def test_point_values_of_linear_fields_are_exact(oracle_mod):
    W, prim_at = _linear_block()
    q = np.moveaxis(W, 0, -1).copy()      # [z][y][x][F] primitive block
    for (x, y, z) in [(3, 3, 3), (5, 8, 4), (10, 10, 10), (2, 7, 9)]:
        for e in DIRS:
            got = oracle_mod.point_value(q, x, y, z, e)
            want = prim_at(x + 0.5 * e[0], y + 0.5 * e[1], z + 0.5 * e[2])
            assert np.max(np.abs(got - want) / np.abs(want)) < 1e-14, (x, y, z, e)


def _face_average(prim_at, centre, d, comp):
    """Average over a unit face (normal d, centre `centre`) of the textbook
    flux components `comp`, by 3x3 Gauss-Legendre (exact up to degree 5 in
    each transverse variable)."""
    t = [k for k in range(3) if k != d]
    gx, gw = np.polynomial.legendre.leggauss(3)
    gx, gw = 0.5 * gx, 0.5 * gw          # nodes and weights on [-1/2, 1/2]
    acc = np.zeros(len(comp))
    for i in range(3):
        for j in range(3):
            p = np.array(centre, dtype=np.float64)
            p[t[0]] += gx[i]
            p[t[1]] += gx[j]
            acc += gw[i] * gw[j] * euler.flux(prim_at(*p), d)[comp]
    return acc


def test_linear_fields_give_the_exact_face_integrals(oracle_mod):
    """Mass and momentum: the flux through a face is at most cubic in the
    transverse coordinates, which Simpson's rule integrates exactly; the
    states on both sides of every point are the exact point values, so the
    central-upwind flux is the physical flux there."""
    n, nf = 8, 11
    W, prim_at = _linear_block(n=n, nf=nf, scale=0.02)
    U = block_from_primitive(W)
    dt, dx = 0.002, 0.05
    out, _ = oracle_mod.step26(U[None], dt=dt, dx=dx)
    lam = dt / dx
    comp = [0, 1, 2, 3]
    err = 0.0
    for z in range(3, 3 + n, 3):
        for y in range(3, 3 + n, 2):
            for x in range(3, 3 + n):
                div = np.zeros(len(comp))
                for d in range(3):
                    c = np.array([x, y, z], dtype=np.float64)
                    cp, cm = c.copy(), c.copy()
                    cp[d] += 0.5
                    cm[d] -= 0.5
                    div += _face_average(prim_at, cp, d, comp) - _face_average(prim_at, cm, d, comp)
                want = U[comp, z, y, x] - lam * div
                got = out[0][comp, z, y, x]
                scale = np.max(np.abs(U[comp]), axis=(1, 2, 3))
                err = max(err, np.max(np.abs(got - want) / scale))
    assert err < 1e-13, err


def test_face_centre_form_is_wrong_for_the_face_integral(oracle_mod):
    """The same linear fields: the face-centre form differs from the exact
    face integrals by the transverse second moment of the momentum flux
    (the term the 26-point form exists to capture), far above rounding."""
    n, nf = 8, 11
    W, prim_at = _linear_block(n=n, nf=nf, scale=0.02)
    U = block_from_primitive(W)
    out6, _ = oracle_mod.step(U[None], dt=0.002, dx=0.05)
    out26, _ = oracle_mod.step26(U[None], dt=0.002, dx=0.05)
    d = normwise(interior(out6[0])[None, 1:4], interior(out26[0])[None, 1:4])
    assert np.max(d) > 1e-12, d


def test_data_varying_along_x_equals_the_face_centre_form(oracle_mod):
    n, nf = 8, 11
    M = n + 6
    U = workloads.random_smooth(1, n=n, nfields=nf, seed=33)
    U[:] = U[:, :, :1, :1, :]              # every (y, z) row the same
    out6, a6 = oracle_mod.step(U, dt=0.003, dx=0.05)
    out26, a26 = oracle_mod.step26(U, dt=0.003, dx=0.05)
    err = normwise(interior(out26), interior(out6))
    assert np.all(err < 1e-14), err
    # the 26 points include the face centres, whose states are those of the
    # face-centre form; the edge and vertex points of y and z faces see the
    # x-edge states, whose signal speeds can only add to the maximum
    assert a26[0] >= a6[0] * (1 - 1e-15)
    # transverse differences vanish exactly: all rows equal bitwise
    I = interior(out26[0])
    assert np.array_equal(I, np.broadcast_to(I[:, :1, :1, :], I.shape))


def test_periodic_brick_conserves_totals(oracle_mod):
    U = workloads.brick(seed=1)
    _, amax = oracle_mod.step26(U, dt=0.0, dx=1 / 64)
    dt = 0.4 * (1 / 64) / amax.max()
    out, _ = oracle_mod.step26(U, dt=dt, dx=1 / 64)
    before, after = fsum_fields(U), fsum_fields(out)
    scale = np.array([math.fsum(np.abs(interior(U)[:, f]).ravel()) for f in range(U.shape[1])])
    assert np.all(np.abs(after - before) <= 1e-13 * scale), (after - before) / scale
    assert np.max(np.abs(interior(out) - interior(U))) > 1e-6


@pytest.mark.parametrize("transform", [_mirror_x, _swap_xy, _swap_xz])
def test_mirror_and_axis_permutation(oracle_mod, transform):
    U = workloads.random_smooth(1, n=8, nfields=11, seed=34)
    dt, dx = 0.003, 0.05
    out, amax = oracle_mod.step26(U, dt=dt, dx=dx)
    out2, amax2 = oracle_mod.step26(transform(U), dt=dt, dx=dx)
    err = normwise(interior(out2), interior(transform(out)))
    assert np.all(err < 1e-14), err
    assert np.allclose(amax2, amax, rtol=1e-15, atol=0)


def test_step26_rejects_bad_arguments(oracle_mod):
    U = workloads.random_smooth(1, n=8, nfields=6, seed=35)
    with pytest.raises(ValueError):
        oracle_mod.step26(U, dt=-1.0, dx=0.1)
    q = np.ones((14, 14, 14, 6))
    with pytest.raises(ValueError):
        oracle_mod.point_value(q, 1, 5, 5, (1, 0, 0))     # stencil leaves the block
    with pytest.raises(ValueError):
        oracle_mod.point_value(q, 5, 5, 5, (0, 0, 0))
