"""Thin ctypes binding of libhydroagg.so (C ABI in include/hydroagg.h).

Argument marshalling only: every step of the hydro path runs in the HIP
kernels of the library.  Device memory and streams come from PyTorch
tensors/streams; they are passed to the library as raw pointers.  If the
library is missing this module raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhydroagg.so")

HYDRO_OK, HYDRO_EINVAL, HYDRO_EHIP, HYDRO_ENOMEM, HYDRO_EAGAIN = 0, -1, -2, -3, -4
GHOST = 3


class HydroError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"hydroagg error {code}: {msg}")
        self.code = code


class hydro_subgrid_t(ctypes.Structure):
    _fields_ = [
        ("u_in", ctypes.c_void_p),
        ("u_out", ctypes.c_void_p),
        ("n", ctypes.c_int32),
        ("nfields", ctypes.c_int32),
        ("level", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


assert ctypes.sizeof(hydro_subgrid_t) == 32

_lib = None


def lib() -> ctypes.CDLL:
    """Load the in-tree library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2210_06438_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER(hydro_subgrid_t)
        for name in ("hydro_step", "hydro_step_each"):
            f = getattr(L, name)
            f.argtypes = [P, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                          ctypes.c_void_p, ctypes.c_void_p]
            f.restype = ctypes.c_int
        L.hydro_plan_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), P, ctypes.c_int32]
        L.hydro_plan_create.restype = ctypes.c_int
        for name in ("hydro_plan_step", "hydro_plan_launch_graph"):
            f = getattr(L, name)
            f.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                          ctypes.c_void_p, ctypes.c_void_p]
            f.restype = ctypes.c_int
        L.hydro_plan_destroy.argtypes = [ctypes.c_void_p]
        L.hydro_plan_destroy.restype = ctypes.c_int
        L.hydro_last_error.argtypes = []
        L.hydro_last_error.restype = ctypes.c_char_p
        L.hydro_version.argtypes = []
        L.hydro_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc: int) -> int:
    if rc != HYDRO_OK:
        raise HydroError(rc, lib().hydro_last_error().decode())
    return rc


def _ptr(t) -> int:
    if t is None:
        return 0
    if isinstance(t, int):
        return t
    return int(t.data_ptr())


def _stream(stream) -> int:
    if stream is None:
        return 0
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def subgrids(u_in, u_out, levels=None, n=None, nfields=None):
    """Descriptor array for a batch stored as float64 tensors
    [count, F, M, M, M] on the GPU (or for explicit lists of pointers)."""
    count = int(u_in.shape[0])
    F = int(u_in.shape[1]) if nfields is None else nfields
    M = int(u_in.shape[2])
    n = M - 2 * GHOST if n is None else n
    if tuple(u_out.shape) != tuple(u_in.shape):
        raise ValueError("u_out must have the shape of u_in")
    if not (u_in.is_contiguous() and u_out.is_contiguous()):
        raise ValueError("tensors must be contiguous")
    stride = F * M * M * M * 8
    arr = (hydro_subgrid_t * max(count, 1))()
    b_in, b_out = _ptr(u_in), _ptr(u_out)
    for s in range(count):
        arr[s].u_in = b_in + s * stride
        arr[s].u_out = b_out + s * stride
        arr[s].n = n
        arr[s].nfields = F
        arr[s].level = 0 if levels is None else int(levels[s])
        arr[s].reserved = 0
    return arr, count


def concat(*descs):
    """Concatenate (array, count) descriptor batches."""
    total = sum(c for _, c in descs)
    arr = (hydro_subgrid_t * max(total, 1))()
    k = 0
    for a, c in descs:
        for i in range(c):
            arr[k] = a[i]
            k += 1
    return arr, total


def hydro_step(descs, dt: float, dx: float, amax=None, stream=None) -> None:
    """Aggregated step: one launch per (n, nfields) class in the batch."""
    arr, count = descs
    _check(lib().hydro_step(arr, count, float(dt), float(dx), _ptr(amax), _stream(stream)))


def hydro_step_each(descs, dt: float, dx: float, amax=None, stream=None) -> None:
    """Baseline: one launch per sub-grid (same kernel)."""
    arr, count = descs
    _check(lib().hydro_step_each(arr, count, float(dt), float(dx), _ptr(amax), _stream(stream)))


def version() -> str:
    return lib().hydro_version().decode()


class Plan:
    """A fixed batch with its descriptor table resident on the device
    (hydro_plan_create); step() launches the kernels, graph() replays them as
    one hipGraph launch.  Keeps the descriptor array alive."""

    def __init__(self, descs):
        self._descs = descs
        arr, count = descs
        self.count = count
        h = ctypes.c_void_p()
        _check(lib().hydro_plan_create(ctypes.byref(h), arr, count))
        self._h = h

    def step(self, dt: float, dx: float, amax=None, stream=None) -> None:
        _check(lib().hydro_plan_step(self._h, float(dt), float(dx), _ptr(amax), _stream(stream)))

    def graph(self, dt: float, dx: float, amax=None, stream=None) -> None:
        _check(lib().hydro_plan_launch_graph(self._h, float(dt), float(dx), _ptr(amax), _stream(stream)))

    def close(self) -> None:
        if self._h:
            _check(lib().hydro_plan_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
