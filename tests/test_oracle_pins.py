"""Pins for the CPU oracle: each test checks it against something the
mathematics or the paper fixes, not against a retyped copy of its formulas.

  uniform state        -> zero update (bitwise), amax = max_d |v_d| + c
  linear primitives    -> the scheme reduces to differences of the exact
                          physical flux at the face centres (textbook Euler
                          flux, tests/ref/euler.py)
  cubic cell averages  -> unlimited PPM interfaces are the exact polynomial
                          values (fourth-order interface formula)
  step in a tracer     -> first-order central-upwind closed forms
  supersonic states    -> the central-upwind flux is the upwind flux
  periodic brick       -> conserved totals change only by rounding
  mirror / permutation -> outputs transform the same way
  contact              -> p and v stay uniform
  uniform composition  -> mass fractions stay uniform
  power-of-two scaling -> bitwise equivariance
  data varying along x -> transverse flux differences vanish exactly: every
                          (y, z) row of the output is the same, bitwise, and
                          zero transverse momentum stays exactly zero
"""
import math

import numpy as np
import pytest

from paper_2210_06438_amd import workloads
from tests.ref import euler

G = 5.0 / 3.0


def block_from_primitive(Wfield):
    """Wfield[F, M, M, M] primitive -> conserved block (independent helper)."""
    return euler.cons(Wfield)


def normwise(a, b):
    """max |a-b| / max |b| per field (fields on axis 0 of the last 4 dims)."""
    a = np.asarray(a)
    b = np.asarray(b)
    nf = a.shape[-4]
    out = []
    for f in range(nf):
        af = a[..., f, :, :, :]
        bf = b[..., f, :, :, :]
        scale = np.max(np.abs(bf))
        out.append(np.max(np.abs(af - bf)) / (scale if scale > 0 else 1.0))
    return np.array(out)


def interior(U, n=8):
    return U[..., 3:3 + n, 3:3 + n, 3:3 + n]


# ---------------------------------------------------------------- uniform
@pytest.mark.parametrize("nf", [6, 11])
@pytest.mark.parametrize("n", [8, 12, 16])
def test_uniform_state_is_a_fixed_point(oracle_mod, n, nf):
    rng = np.random.default_rng(10 + n + nf)
    M = n + 6
    for trial in range(3):
        rho, p = rng.uniform(0.1, 5.0, size=2)
        v = rng.uniform(-2.0, 2.0, size=3)
        W = np.concatenate([[rho], v, [p], rng.uniform(0.1, 1.0, size=nf - 5)])
        U = np.broadcast_to(euler.cons(W)[:, None, None, None], (nf, M, M, M)).copy()
        out, amax = oracle_mod.step(U[None], dt=0.37, dx=0.01)
        assert np.array_equal(out[0], U)
        expect = max(abs(v[d]) for d in range(3)) + math.sqrt(G * p / rho)
        assert abs(amax[0] - expect) <= 1e-14 * expect


# ---------------------------------------------------------------- linear
@pytest.mark.parametrize("axes", [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 1)])
def test_linear_primitives_reduce_to_exact_face_fluxes(oracle_mod, axes):
    """With every primitive linear in the cell index, PPM returns the exact
    face-centre values on both sides of every face (no limiter fires), the
    central-upwind flux of two equal states is the physical flux, and the
    update is U - lambda * sum_d [F_d(W(face+)) - F_d(W(face-))]."""
    n, nf = 8, 11
    M = n + 6
    rng = np.random.default_rng(7)
    base = np.array([1.0, 0.3, -0.2, 0.1, 2.0, 0.5, 0.1, 0.2, 0.3, 0.25, 0.15])
    grad = rng.uniform(-1.0, 1.0, size=(nf, 3)) * 0.01 * np.abs(base)[:, None]
    grad *= np.array(axes)[None, :]
    grid = np.arange(M, dtype=np.float64)

    def prim_at(x, y, z):
        return base[:, None] + grad[:, 0:1] * x + grad[:, 1:2] * y + grad[:, 2:3] * z

    Z, Y, X = np.meshgrid(grid, grid, grid, indexing="ij")
    W = prim_at(X.ravel(), Y.ravel(), Z.ravel()).reshape(nf, M, M, M)
    U = block_from_primitive(W)
    dt, dx = 0.002, 0.05
    out, _ = oracle_mod.step(U[None], dt=dt, dx=dx)
    lam = dt / dx
    expect = U.copy()
    for z in range(3, 3 + n):
        for y in range(3, 3 + n):
            for x in range(3, 3 + n):
                div = np.zeros(nf)
                for d in range(3):
                    e = np.zeros(3)
                    e[d] = 0.5
                    Wp = prim_at(x + e[0], y + e[1], z + e[2])[:, 0]
                    Wm = prim_at(x - e[0], y - e[1], z - e[2])[:, 0]
                    div += euler.flux(Wp, d) - euler.flux(Wm, d)
                expect[:, z, y, x] = U[:, z, y, x] - lam * div
    err = normwise(interior(out[0]), interior(expect))
    assert np.all(err < 1e-13), err


# ---------------------------------------------------------------- cubic
def _cubic_averages(coef, centres, h=1.0):
    """Cell averages of P(x) = sum coef[k] x^k over [c - h/2, c + h/2]."""
    def Q(x):
        return sum(c * x ** (k + 1) / (k + 1) for k, c in enumerate(coef))
    return (Q(centres + h / 2) - Q(centres - h / 2)) / h


def _poly(coef, x):
    return sum(c * x ** k for k, c in enumerate(coef))


def test_ppm_interfaces_are_exact_for_cubic_averages(oracle_mod):
    coef = [1.0, 0.3, 0.02, 0.001]       # monotone, mildly curved on [0, 14]
    centres = np.arange(14, dtype=np.float64)
    q = _cubic_averages(coef, centres)
    qL, qR, cnt = oracle_mod.ppm_line(q, counters=True)
    assert cnt["slope_limited"] == 0 and cnt["slope_zero"] == 0
    assert cnt["par_keep"] == 10 and cnt["par_flat"] == cnt["par_left"] == cnt["par_right"] == 0
    for i in range(2, 12):
        assert abs(qL[i, 0] - _poly(coef, i - 0.5)) < 1e-13
        assert abs(qR[i, 0] - _poly(coef, i + 0.5)) < 1e-13


def test_tracer_with_cubic_profile_is_advected_at_fourth_order(oracle_mod):
    """Uniform flow; tau = cell averages of a cubic in x.  Each face then
    carries tau(face) * v exactly, so tau_out = tau - lambda v (P(x+1/2) -
    P(x-1/2))."""
    n, nf = 8, 6
    M = n + 6
    coef = [2.0, 0.1, 0.004, 0.0002]
    tau_line = _cubic_averages(coef, np.arange(M, dtype=np.float64))
    for v in (0.3, 2.5):                  # subsonic and supersonic
        W = np.zeros((nf, M, M, M))
        W[0], W[1], W[4] = 1.0, v, 1.0
        W[5] = tau_line[None, None, :]
        U = block_from_primitive(W)
        dt, dx = 0.01, 0.1
        out, _ = oracle_mod.step(U[None], dt=dt, dx=dx)
        lam = dt / dx
        x = np.arange(3, 3 + n, dtype=np.float64)
        expect = tau_line[3:3 + n] - lam * v * (_poly(coef, x + 0.5) - _poly(coef, x - 0.5))
        got = out[0, 5, 3:3 + n, 3:3 + n, 3:3 + n]
        assert np.max(np.abs(got - expect[None, None, :])) < 1e-13
        # hydro fields of a uniform flow are untouched
        assert np.array_equal(out[0, :5], U[:5])


# ---------------------------------------------------------------- step
@pytest.mark.parametrize("v", [0.3, -0.4, 2.0])
def test_tracer_step_closed_form(oracle_mod, v):
    """tau = A left of the face between stored x=6 and 7, B right of it.
    All slopes vanish, both neighbouring parabolas flatten, and the face sees
    W- = A, W+ = B with a+ = max(v + c, 0), a- = min(v - c, 0):
    subsonic: tau(6) = A - lambda/2 (v - c)(B - A), tau(7) = B - lambda/2 (v + c)(B - A);
    supersonic (a- = 0): tau(6) = A, tau(7) = B - lambda v (B - A)."""
    n, nf = 8, 6
    M = n + 6
    A, B = 0.7, 1.9
    W = np.zeros((nf, M, M, M))
    W[0], W[1], W[4] = 1.0, v, 1.0
    W[5] = np.where(np.arange(M) <= 6, A, B)[None, None, :]
    U = block_from_primitive(W)
    dt, dx = 0.01, 0.1
    lam = dt / dx
    out, amax = oracle_mod.step(U[None], dt=dt, dx=dx)
    c = math.sqrt(G)
    ap, am = max(v + c, 0.0), min(v - c, 0.0)
    tau = out[0, 5, 3:11, 3:11, :]
    if am < 0 and ap > 0:
        e6 = A - 0.5 * lam * (v - c) * (B - A)
        e7 = B - 0.5 * lam * (v + c) * (B - A)
    else:
        assert ap > 0
        e6 = A
        e7 = B - lam * v * (B - A)
    assert np.max(np.abs(tau[..., 6] - e6)) < 1e-14
    assert np.max(np.abs(tau[..., 7] - e7)) < 1e-14
    for x in (3, 4, 5, 8, 9, 10):
        assert np.max(np.abs(tau[..., x] - (A if x <= 6 else B))) < 1e-14
    assert abs(amax[0] - max(ap, -am)) < 1e-15 * max(ap, -am)


# ---------------------------------------------------------------- flux limits
def _rand_state(rng, nf=11, vlo=-1.0, vhi=1.0):
    return np.concatenate([[rng.uniform(0.2, 3.0)], rng.uniform(vlo, vhi, 3),
                           [rng.uniform(0.2, 3.0)], rng.uniform(0.0, 1.0, nf - 5)])


def test_central_upwind_flux_limits(oracle_mod):
    rng = np.random.default_rng(3)
    for _ in range(50):
        d = int(rng.integers(3))
        W = _rand_state(rng)
        F, s = oracle_mod.knp_flux(W, W, d)
        ref = euler.flux(W, d)
        assert np.max(np.abs(F - ref)) <= 1e-14 * np.max(np.abs(ref))
        c = euler.sound_speed(W)
        assert abs(s - (abs(W[1 + d]) + c)) <= 1e-15 * (abs(W[1 + d]) + c)
        # supersonic towards +d: the flux is the low-side physical flux
        Wm, Wp = _rand_state(rng), _rand_state(rng)
        Wm[1 + d] = euler.sound_speed(Wm) + rng.uniform(0.01, 1.0)
        Wp[1 + d] = euler.sound_speed(Wp) + rng.uniform(0.01, 1.0)
        F, s = oracle_mod.knp_flux(Wm, Wp, d)
        ref = euler.flux(Wm, d)
        assert np.max(np.abs(F - ref)) <= 1e-14 * np.max(np.abs(ref))
        assert s == pytest.approx(max(Wm[1 + d] + euler.sound_speed(Wm),
                                      Wp[1 + d] + euler.sound_speed(Wp)), rel=1e-15)
        # supersonic towards -d: the high-side physical flux
        Wm[1 + d] = -euler.sound_speed(Wm) - rng.uniform(0.01, 1.0)
        Wp[1 + d] = -euler.sound_speed(Wp) - rng.uniform(0.01, 1.0)
        F, _ = oracle_mod.knp_flux(Wm, Wp, d)
        ref = euler.flux(Wp, d)
        assert np.max(np.abs(F - ref)) <= 1e-14 * np.max(np.abs(ref))


def test_central_upwind_symmetric_speeds_is_rusanov(oracle_mod):
    """Two states at rest with equal sound speed: a+ = -a- = c and the flux is
    (F- + F+)/2 - c/2 (U+ - U-)."""
    rng = np.random.default_rng(4)
    for d in range(3):
        r1, r2 = rng.uniform(0.5, 2.0, 2)
        Wm = np.array([r1, 0, 0, 0, 0.7 * r1, 0.3])
        Wp = np.array([r2, 0, 0, 0, 0.7 * r2, 0.9])
        c = math.sqrt(G * 0.7)
        F, s = oracle_mod.knp_flux(Wm, Wp, d)
        ref = 0.5 * (euler.flux(Wm, d) + euler.flux(Wp, d)) - 0.5 * c * (euler.cons(Wp) - euler.cons(Wm))
        assert np.max(np.abs(F - ref)) < 1e-14
        assert s == pytest.approx(c, rel=1e-15)


# ---------------------------------------------------------------- PPM properties
def test_ppm_limited_parabolas_are_monotone(oracle_mod):
    rng = np.random.default_rng(5)
    seen = {"par_left": 0, "par_right": 0, "par_flat": 0, "par_keep": 0, "slope_limited": 0}
    for _ in range(300):
        q = np.cumsum(rng.normal(size=14)) + rng.normal(size=14) * rng.uniform(0, 2)
        qL, qR, cnt = oracle_mod.ppm_line(q, counters=True)
        for k in seen:
            seen[k] += cnt[k]
        for i in range(2, 12):
            l, r, c = qL[i, 0], qR[i, 0], q[i]
            lo, hi = min(q[i - 1:i + 2]), max(q[i - 1:i + 2])
            assert lo - 1e-12 <= l <= hi + 1e-12 and lo - 1e-12 <= r <= hi + 1e-12
            if l == r == c:
                continue
            assert (r - c) * (c - l) > 0
            q6 = 6.0 * (c - 0.5 * (l + r))
            assert abs(q6) <= abs(r - l) * (1 + 1e-12) + 1e-12
            # a strict local extremum always flattens
            if (q[i] - q[i - 1]) * (q[i + 1] - q[i]) < 0:
                raise AssertionError("extremum not flattened")
    assert all(v > 0 for v in seen.values()), seen


def test_ppm_overshoot_fix_puts_the_extremum_on_the_edge(oracle_mod):
    """When the limiter resets one edge it makes the parabola's derivative
    vanish at that edge: q6 = +-(qR - qL) exactly (up to rounding)."""
    q = np.array([0.0, 0.0, 0.0, 0.0, 0.1, 1.0, 1.02, 1.02, 1.02, 1.02, 1.02, 1.02, 1.02, 1.02])
    qL, qR, cnt = oracle_mod.ppm_line(q, counters=True)
    assert cnt["par_left"] + cnt["par_right"] > 0
    fixed = 0
    for i in range(2, 12):
        l, r, c = qL[i, 0], qR[i, 0], q[i]
        if l == r == c:
            continue
        q6 = 6.0 * (c - 0.5 * (l + r))
        if abs(abs(q6) - abs(r - l)) <= 1e-12:
            fixed += 1
    assert fixed >= cnt["par_left"] + cnt["par_right"]


def test_ppm_step_is_first_order(oracle_mod):
    q = np.array([1.0] * 7 + [3.0] * 7)
    qL, qR = oracle_mod.ppm_line(q)
    for i in range(2, 12):
        assert qL[i, 0] == q[i] and qR[i, 0] == q[i]


# ---------------------------------------------------------------- invariants
def fsum_fields(U, n=8):
    Ui = U[..., 3:3 + n, 3:3 + n, 3:3 + n]
    return np.array([math.fsum(Ui[:, f].ravel()) for f in range(U.shape[1])])


def test_periodic_brick_conserves_totals(oracle_mod):
    U = workloads.brick(seed=1)
    _, amax = oracle_mod.step(U, dt=0.0, dx=1 / 64)
    dt = 0.4 * (1 / 64) / amax.max()
    out, _ = oracle_mod.step(U, dt=dt, dx=1 / 64)
    before, after = fsum_fields(U), fsum_fields(out)
    scale = np.array([math.fsum(np.abs(interior(U)[:, f]).ravel()) for f in range(U.shape[1])])
    assert np.all(np.abs(after - before) <= 1e-13 * scale), (after - before) / scale
    # and the step did something
    assert np.max(np.abs(interior(out) - interior(U))) > 1e-6


def test_dt_zero_copies_interior_and_leaves_ghosts(oracle_mod):
    U = workloads.random_smooth(2, n=8, nfields=11, seed=9)
    sentinel = np.full_like(U, np.nan)
    out, amax = oracle_mod.step(U, dt=0.0, dx=0.1, u_out=sentinel)
    assert np.array_equal(interior(out), interior(U))
    ghost = np.ones(U.shape[2:], dtype=bool)
    ghost[3:11, 3:11, 3:11] = False
    assert np.all(np.isnan(out[:, :, ghost]))
    assert np.all(amax > 0)


def _mirror_x(U):
    V = U[..., ::-1].copy()
    V[:, 1] *= -1.0
    return V


def _swap_xy(U):
    V = np.swapaxes(U, -1, -2).copy()
    V[:, [1, 2]] = V[:, [2, 1]]
    return V


def _swap_xz(U):
    V = np.swapaxes(U, -1, -3).copy()
    V[:, [1, 3]] = V[:, [3, 1]]
    return V


@pytest.mark.parametrize("transform", [_mirror_x, _swap_xy, _swap_xz])
def test_mirror_and_axis_permutation(oracle_mod, transform):
    U = workloads.random_smooth(2, n=8, nfields=11, seed=11)
    dt, dx = 0.003, 0.05
    out, amax = oracle_mod.step(U, dt=dt, dx=dx)
    out2, amax2 = oracle_mod.step(transform(U), dt=dt, dx=dx)
    err = normwise(interior(out2), interior(transform(out)))
    assert np.all(err < 1e-14), err
    assert np.allclose(amax2, amax, rtol=1e-15, atol=0)


def test_contact_keeps_pressure_and_velocity_uniform(oracle_mod):
    n, nf = 8, 11
    M = n + 6
    rng = np.random.default_rng(12)
    W = np.empty((nf, M, M, M))
    W[0] = rng.uniform(0.5, 2.0, (M, M, M))
    W[1], W[2], W[3], W[4] = 0.2, -0.1, 0.05, 1.3
    W[5:] = rng.uniform(0.1, 1.0, (nf - 5, M, M, M))
    U = block_from_primitive(W)
    _, amax = oracle_mod.step(U[None], dt=0.0, dx=0.1)
    out, _ = oracle_mod.step(U[None], dt=0.4 * 0.1 / amax[0], dx=0.1)
    Ui = interior(out[0])
    rho = Ui[0]
    v = Ui[1:4] / rho
    p = (G - 1) * (Ui[4] - 0.5 * (Ui[1] * v[0] + Ui[2] * v[1] + Ui[3] * v[2]))
    assert np.max(np.abs(v[0] - 0.2)) < 1e-13
    assert np.max(np.abs(v[1] + 0.1)) < 1e-13
    assert np.max(np.abs(v[2] - 0.05)) < 1e-13
    assert np.max(np.abs(p - 1.3)) < 1e-13 * 1.3
    assert np.max(np.abs(rho - interior(U)[0])) > 1e-3   # the density moved


def test_uniform_composition_stays_uniform(oracle_mod):
    U = workloads.random_smooth(2, n=8, nfields=11, seed=13)
    X = np.array([0.1, 0.2, 0.3, 0.15, 0.25])
    U[:, 6:11] = U[:, 0:1] * X[None, :, None, None, None]
    out, _ = oracle_mod.step(U, dt=0.004, dx=0.05)
    frac = interior(out)[:, 6:11] / interior(out)[:, 0:1]
    assert np.max(np.abs(frac - X[None, :, None, None, None])) < 1e-14


def test_power_of_two_scaling_is_bitwise(oracle_mod):
    U = workloads.random_smooth(3, n=8, nfields=11, seed=14)
    dt, dx = 0.004, 0.05
    out, amax = oracle_mod.step(U, dt=dt, dx=dx, levels=[0, 1, 2])
    out2, amax2 = oracle_mod.step(2.0 * U, dt=dt, dx=dx, levels=[0, 1, 2])
    assert np.array_equal(interior(out2), 2.0 * interior(out))
    assert np.array_equal(amax2, amax)
    out3, amax3 = oracle_mod.step(U, dt=2 * dt, dx=2 * dx, levels=[0, 1, 2])
    assert np.array_equal(interior(out3), interior(out))
    assert np.array_equal(amax3, amax)


def test_level_halves_the_cell_width(oracle_mod):
    U = workloads.random_smooth(1, n=8, nfields=6, seed=15)
    a, _ = oracle_mod.step(U, dt=0.002, dx=0.1, levels=[1])
    b, _ = oracle_mod.step(U, dt=0.004, dx=0.1, levels=[0])
    assert np.array_equal(interior(a), interior(b))


def test_threaded_oracle_matches_sequential(oracle_mod):
    U = workloads.random_smooth(6, n=8, nfields=11, seed=16)
    a, aa = oracle_mod.step(U, dt=0.003, dx=0.05)
    b, bb = oracle_mod.step(U, dt=0.003, dx=0.05, nthreads=4)
    assert np.array_equal(a, b) and np.array_equal(aa, bb)


def test_oracle_rejects_bad_arguments(oracle_mod):
    U = workloads.random_smooth(1, n=8, nfields=6, seed=1)
    with pytest.raises(ValueError):
        oracle_mod.step(U, dt=-1.0, dx=0.1)
    with pytest.raises(ValueError):
        oracle_mod.step(U, dt=0.1, dx=0.0)
    with pytest.raises(ValueError):
        oracle_mod.step(U[:, :, :10], dt=0.1, dx=0.1)


# ------------------------------------------------- one-dimensional data
def x_only_block(n, nf, seed):
    """A block whose primitives vary only along x (v_y = v_z = 0)."""
    M = n + 6
    rng = np.random.default_rng(seed)
    W = np.empty((nf, M))
    W[0] = 1.0 + 0.3 * rng.uniform(-1, 1, M)
    W[1] = 0.4 * rng.uniform(-1, 1, M)
    W[2] = W[3] = 0.0
    W[4] = 1.0 + 0.3 * rng.uniform(-1, 1, M)
    for f in range(5, nf):
        W[f] = W[0] * rng.uniform(0.05, 0.3, M)
    Wf = np.broadcast_to(W[:, None, None, :], (nf, M, M, M)).copy()
    return block_from_primitive(Wf)


@pytest.mark.parametrize("n,nf", [(8, 11), (12, 6), (16, 11)])
def test_x_only_data_has_no_transverse_update(oracle_mod, n, nf):
    U = x_only_block(n, nf, seed=n + nf)[None]
    out, amax = oracle_mod.step(U, 0.002, 0.05)
    I = interior(out, n)[0]
    # identical rows along y and z
    assert np.array_equal(I, np.broadcast_to(I[:, :1, :1, :], I.shape))
    # transverse momenta exactly zero, and the x update is not trivial
    assert not I[2].any() and not I[3].any()
    assert not np.array_equal(I, interior(U, n)[0])
