"""CPU FP64 oracle for the sub-grid hydro step -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product (``paper_2210_06438_amd``)
never does, and the two share no code: the oracle is plain C in
``hydro_oracle.c`` (built with gcc, ``-ffp-contract=off``), wrapped here with
ctypes and numpy.

What it computes is one forward-Euler stage of the ideal-gas Euler step on
N^3 sub-grids with 3 ghost layers (Section IV-B of the paper: PPM
reconstruction, central-upwind fluxes at the face centres, flux-divergence
update; Section V-A: sub-grid shape).  Every function below names the step it
follows; the C file restates each step.

Parity status: pinned by the CPU tests under ``tests/test_oracle_*.py``
(uniform state, linear and cubic closed forms, discontinuity closed forms,
conservation, symmetry, contact preservation, scaling, Sod convergence to the
exact Riemann solution).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hydro_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

GAMMA = 5.0 / 3.0
GHOST = 3
COUNTER_NAMES = (
    "slope_zero", "slope_central", "slope_limited",
    "par_flat", "par_left", "par_right", "par_keep",
    "nonpos_cell", "nonpos_face",
)


class _Subgrid(ctypes.Structure):
    _fields_ = [
        ("u_in", ctypes.c_void_p),
        ("u_out", ctypes.c_void_p),
        ("n", ctypes.c_int32),
        ("nfields", ctypes.c_int32),
        ("level", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/liboracle.so``."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-fopenmp", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_step.argtypes = [ctypes.POINTER(_Subgrid), ctypes.c_int,
                                    ctypes.c_double, ctypes.c_double, dp, i64p,
                                    ctypes.c_int]
        lib.oracle_step.restype = ctypes.c_int
        lib.oracle_step26.argtypes = lib.oracle_step.argtypes
        lib.oracle_step26.restype = ctypes.c_int
        lib.oracle_point_value.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int, ctypes.c_int,
                                           ctypes.POINTER(ctypes.c_int32), dp]
        lib.oracle_point_value.restype = ctypes.c_int
        lib.oracle_primitive.argtypes = [dp, ctypes.c_int, dp]
        lib.oracle_primitive.restype = None
        lib.oracle_ppm_line.argtypes = [dp, ctypes.c_int, ctypes.c_int, dp, dp, i64p]
        lib.oracle_ppm_line.restype = ctypes.c_int
        lib.oracle_state.argtypes = [dp, ctypes.c_int, dp]
        lib.oracle_state.restype = None
        lib.oracle_flux.argtypes = [dp, ctypes.c_int, ctypes.c_int, dp]
        lib.oracle_flux.restype = None
        lib.oracle_knp_flux.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, dp]
        lib.oracle_knp_flux.restype = ctypes.c_double
        lib.oracle_max_threads.argtypes = []
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def step26(u_in: np.ndarray, dt: float, dx: float, levels=None, u_out=None,
           counters: bool = False, nthreads: int = 1):
    """Q1-Q7: the 26-point form (values at the 26 points of each cell's
    surface, central-upwind fluxes at the 9 points of every face, Simpson's
    rule over each face), with the arguments and results of step().  The
    sub-grids' edge and corner ghosts are read."""
    return step(u_in, dt, dx, levels=levels, u_out=u_out, counters=counters,
                nthreads=nthreads, _points=26)


def point_value(q_block, x: int, y: int, z: int, e):
    """Q2+Q3: the value of stored cell (x, y, z) of a block of primitives
    q_block[M, M, M, F] toward direction e (three of -1, 0, 1)."""
    lib = _load()
    q = _f64(q_block)
    M, nf = q.shape[0], q.shape[3]
    ev = (ctypes.c_int32 * 3)(*[int(v) for v in e])
    out = np.empty(nf, dtype=np.float64)
    if lib.oracle_point_value(_dp(q), M, nf, int(x), int(y), int(z), ev, _dp(out)) != 0:
        raise ValueError("stencil outside the block or bad direction")
    return out


def step(u_in: np.ndarray, dt: float, dx: float, levels=None, u_out=None,
         counters: bool = False, nthreads: int = 1, _points: int = 6):
    """O1-O7 on a batch of sub-grids.

    ``u_in``: float64 array [count, F, M, M, M] (M = N + 6), SoA, x fastest.
    ``levels``: per-sub-grid octree level (dx_s = dx * 2**-level), default 0.
    ``u_out``: optional array of the same shape; only interior cells are
    written (ghosts keep whatever ``u_out`` held, a copy of ``u_in`` if None).
    Returns ``(u_out, amax[count])`` or ``(u_out, amax, counters_dict)``.
    """
    lib = _load()
    u_in = _f64(u_in)
    if u_in.ndim != 5:
        raise ValueError("u_in must be [count, F, M, M, M]")
    count, nf, M = u_in.shape[0], u_in.shape[1], u_in.shape[2]
    if not (u_in.shape[2] == u_in.shape[3] == u_in.shape[4]) or M <= 2 * GHOST:
        raise ValueError("sub-grids must be cubes with edge > 6")
    n = M - 2 * GHOST
    if u_out is None:
        u_out = u_in.copy()
    else:
        if u_out.shape != u_in.shape or u_out.dtype != np.float64 or not u_out.flags.c_contiguous:
            raise ValueError("u_out must be a C-contiguous float64 array like u_in")
    if levels is None:
        levels = np.zeros(count, dtype=np.int64)
    levels = np.asarray(levels, dtype=np.int64).reshape(count)
    descs = (_Subgrid * max(count, 1))()
    stride = nf * M * M * M * 8
    for s in range(count):
        descs[s].u_in = u_in.ctypes.data + s * stride
        descs[s].u_out = u_out.ctypes.data + s * stride
        descs[s].n = n
        descs[s].nfields = nf
        descs[s].level = int(levels[s])
        descs[s].reserved = 0
    amax = np.zeros(max(count, 1), dtype=np.float64)
    cnt = np.zeros(len(COUNTER_NAMES), dtype=np.int64)
    fn = lib.oracle_step26 if _points == 26 else lib.oracle_step
    rc = fn(descs, count, float(dt), float(dx), _dp(amax),
            cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) if counters else None,
            int(nthreads))
    if rc != 0:
        raise ValueError("oracle step rejected its arguments")
    amax = amax[:count]
    if counters:
        return u_out, amax, dict(zip(COUNTER_NAMES, (int(c) for c in cnt)))
    return u_out, amax


def primitive(U) -> np.ndarray:
    """O1 on one cell: conserved U[F] -> primitive q[F]."""
    lib = _load()
    U = _f64(U)
    q = np.empty_like(U)
    lib.oracle_primitive(_dp(U), U.shape[0], _dp(q))
    return q


def ppm_line(q, counters: bool = False):
    """O2-O3 on one line q[len, F]; returns (qL, qR) with NaN where unset
    (only cells 2..len-3 are reconstructed)."""
    lib = _load()
    q = _f64(q)
    if q.ndim == 1:
        q = q[:, None]
    L, nf = q.shape
    qL = np.full_like(q, np.nan)
    qR = np.full_like(q, np.nan)
    cnt = np.zeros(len(COUNTER_NAMES), dtype=np.int64)
    rc = lib.oracle_ppm_line(_dp(q), L, nf, _dp(qL), _dp(qR),
                             cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if rc != 0:
        raise ValueError("bad line")
    if counters:
        return qL, qR, dict(zip(COUNTER_NAMES, (int(c) for c in cnt)))
    return qL, qR


def state(W) -> np.ndarray:
    """O5: conserved state of a primitive state W[F]."""
    lib = _load()
    W = _f64(W)
    U = np.empty_like(W)
    lib.oracle_state(_dp(W), W.shape[0], _dp(U))
    return U


def flux(W, d: int) -> np.ndarray:
    """O5: physical flux along axis d of a primitive state W[F]."""
    lib = _load()
    W = _f64(W)
    F = np.empty_like(W)
    lib.oracle_flux(_dp(W), W.shape[0], int(d), _dp(F))
    return F


def knp_flux(Wm, Wp, d: int):
    """O6: central-upwind flux between primitive states Wm (low side) and Wp
    (high side) along axis d.  Returns (Fhat[F], max(a+, -a-))."""
    lib = _load()
    Wm = _f64(Wm)
    Wp = _f64(Wp)
    if Wm.shape != Wp.shape or Wm.shape[0] > 16:
        raise ValueError("states must have the same length <= 16")
    F = np.empty_like(Wm)
    s = lib.oracle_knp_flux(_dp(Wm), _dp(Wp), Wm.shape[0], int(d), _dp(F))
    return F, float(s)


def max_threads() -> int:
    return int(_load().oracle_max_threads())
