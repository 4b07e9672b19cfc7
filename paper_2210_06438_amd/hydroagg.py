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
OUT_STORED = 0      # u_out in the (n+6)^3 layout of u_in, interior written
OUT_INTERIOR = 1    # u_out holds the interior only, [F][n][n][n]
STATIC_MAX = 8192   # most sub-grids of one hydro_step_static call


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
        ("out_layout", ctypes.c_int32),
    ]


assert ctypes.sizeof(hydro_subgrid_t) == 32


class hydro_agg_stats_t(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "submitted", "batches", "launched", "flush_width", "flush_idle", "flush_timeout",
        "flush_manual", "refused")] + [("width_hist", ctypes.c_uint64 * 11),
                                       ("held", ctypes.c_uint64), ("held_bytes", ctypes.c_uint64)]

    def as_dict(self):
        d = {n: int(getattr(self, n)) for n, _ in self._fields_ if n != "width_hist"}
        d["width_hist"] = [int(x) for x in self.width_hist]
        return d


class hydro_serve_config_t(ctypes.Structure):
    _fields_ = [("max_width", ctypes.c_int32), ("timeout_us", ctypes.c_double),
                ("n_streams", ctypes.c_int32), ("flush_when_idle", ctypes.c_int32),
                ("nfields", ctypes.c_int32), ("dt", ctypes.c_double), ("dx", ctypes.c_double),
                ("slab_base", ctypes.c_void_p * 3), ("slabs", ctypes.c_int32 * 3),
                ("keep_slabs", ctypes.c_int32), ("out_layout", ctypes.c_int32)]


class hydro_serve_stats_t(ctypes.Structure):
    _fields_ = [("agg", hydro_agg_stats_t), ("makespan_us", ctypes.c_double),
                ("first_admit_us", ctypes.c_double), ("max_live", ctypes.c_uint64),
                ("slab_waits", ctypes.c_uint64), ("launch_host_us", ctypes.c_double)]

class hydro_brick_t(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nfields", ctypes.c_int32), ("nb", ctypes.c_int32 * 3),
                ("bc", ctypes.c_int32 * 3), ("level", ctypes.c_int32)]


BC_PERIODIC = 0
BC_OUTFLOW = 1


class hydro_region_task_t(ctypes.Structure):
    _fields_ = [("team", ctypes.c_int32), ("index", ctypes.c_int32), ("size", ctypes.c_int32),
                ("stream", ctypes.c_int32), ("id", ctypes.c_uint64)]


class hydro_region_stats_t(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "tasks", "teams", "full_teams", "uploads", "launches", "downloads")] + \
        [("size_hist", ctypes.c_uint64 * 11)]


class hydro_region_axpby_t(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("out", ctypes.c_void_p),
                ("a", ctypes.c_double), ("b", ctypes.c_double), ("n", ctypes.c_int64)]


REGION_STEP8_F6, REGION_STEP8_F11, REGION_AXPBY = 0, 1, 2
DRIVE_REGION, DRIVE_EACH = 0, 1

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
        for name in ("hydro_step", "hydro_step_each", "hydro_step_static", "hydro_step26"):
            f = getattr(L, name)
            f.argtypes = [P, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                          ctypes.c_void_p, ctypes.c_void_p]
            f.restype = ctypes.c_int
        L.hydro_plan_pattern_floor.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]
        L.hydro_plan_pattern_floor.restype = ctypes.c_int
        L.hydro_plan_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), P, ctypes.c_int32]
        L.hydro_plan_create.restype = ctypes.c_int
        for name in ("hydro_plan_step", "hydro_plan_launch_graph"):
            f = getattr(L, name)
            f.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                          ctypes.c_void_p, ctypes.c_void_p]
            f.restype = ctypes.c_int
        L.hydro_plan_destroy.argtypes = [ctypes.c_void_p]
        L.hydro_plan_destroy.restype = ctypes.c_int
        AP = ctypes.c_void_p
        L.hydro_agg_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, ctypes.c_double,
                                       ctypes.c_int32, ctypes.c_uint64, ctypes.c_int32]
        L.hydro_submit.argtypes = [AP, P, ctypes.c_double, ctypes.c_double, ctypes.POINTER(ctypes.c_uint64)]
        L.hydro_submit_many.argtypes = [AP, P, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]
        L.hydro_agg_drain.argtypes = [AP]
        L.hydro_step_streams.argtypes = [P, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]
        RT = ctypes.POINTER(hydro_region_task_t)
        VP = ctypes.c_void_p
        L.hydro_region_create.argtypes = [ctypes.POINTER(VP), ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_uint64]
        L.hydro_region_enter.argtypes = [VP, RT]
        L.hydro_region_alloc.argtypes = [VP, RT, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(VP), ctypes.POINTER(VP)]
        L.hydro_region_buffer.argtypes = [VP, RT, ctypes.c_int32, ctypes.POINTER(VP),
                                          ctypes.POINTER(ctypes.c_uint64)]
        L.hydro_region_upload.argtypes = [VP, RT, ctypes.c_int32]
        L.hydro_region_download.argtypes = [VP, RT, ctypes.c_int32]
        L.hydro_region_launch.argtypes = [VP, RT, VP, ctypes.c_uint32, ctypes.c_uint32,
                                          ctypes.c_uint32, ctypes.POINTER(VP)]
        L.hydro_region_wait.argtypes = [VP, RT]
        L.hydro_region_leave.argtypes = [VP, RT]
        L.hydro_region_drive.argtypes = [VP, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_double)]
        L.hydro_region_stats.argtypes = [VP, ctypes.POINTER(hydro_region_stats_t)]
        L.hydro_region_destroy.argtypes = [VP]
        for name in ("hydro_region_create", "hydro_region_enter", "hydro_region_alloc",
                     "hydro_region_buffer", "hydro_region_upload", "hydro_region_download",
                     "hydro_region_launch", "hydro_region_wait", "hydro_region_leave",
                     "hydro_region_stats", "hydro_region_destroy", "hydro_region_drive"):
            getattr(L, name).restype = ctypes.c_int
        L.hydro_region_kernel.argtypes = [ctypes.c_int32]
        L.hydro_region_kernel.restype = VP
        L.hydro_flush.argtypes = [AP]
        L.hydro_progress.argtypes = [AP]
        L.hydro_poll.argtypes = [AP, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32),
                                 ctypes.POINTER(ctypes.c_double)]
        L.hydro_wait.argtypes = [AP, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)]
        L.hydro_agg_stats.argtypes = [AP, ctypes.POINTER(hydro_agg_stats_t)]
        L.hydro_agg_destroy.argtypes = [AP]
        L.hydro_serve_run.argtypes = [ctypes.POINTER(hydro_serve_config_t), P, ctypes.c_int32,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.POINTER(hydro_serve_stats_t)]
        for name in ("hydro_agg_create", "hydro_submit", "hydro_flush", "hydro_progress",
                     "hydro_poll", "hydro_wait", "hydro_agg_stats", "hydro_agg_destroy",
                     "hydro_serve_run", "hydro_submit_many", "hydro_agg_drain",
                     "hydro_step_streams"):
            getattr(L, name).restype = ctypes.c_int
        L.hydro_set_tile.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        L.hydro_set_tile.restype = ctypes.c_int
        L.hydro_get_tile.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
        L.hydro_get_tile.restype = ctypes.c_int
        BP = ctypes.POINTER(hydro_brick_t)
        L.hydro_ghost_fill.argtypes = [BP, ctypes.c_void_p, ctypes.c_void_p]
        L.hydro_ghost_fill_faces.argtypes = [BP, ctypes.c_void_p, ctypes.c_void_p]
        L.hydro_rk3_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), BP, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p]
        L.hydro_rk3_stage.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]
        for name in ("hydro_rk3_step", "hydro_rk3_launch_graph"):
            getattr(L, name).argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_void_p, ctypes.c_void_p]
        L.hydro_rk3_destroy.argtypes = [ctypes.c_void_p]
        for name in ("hydro_ghost_fill", "hydro_ghost_fill_faces", "hydro_rk3_create",
                     "hydro_rk3_stage", "hydro_rk3_step",
                     "hydro_rk3_launch_graph", "hydro_rk3_destroy"):
            getattr(L, name).restype = ctypes.c_int
        L.hydro_math_check.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p]
        L.hydro_math_check.restype = ctypes.c_int
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


def set_tile(n, nfields, tile):
    """Step sub-grids of class (n, nfields) as tile^3 blocks (4 or 8)."""
    _check(lib().hydro_set_tile(int(n), int(nfields), int(tile)))


def get_tile(n, nfields):
    t = ctypes.c_int32()
    _check(lib().hydro_get_tile(int(n), int(nfields), ctypes.byref(t)))
    return int(t.value)


def subgrids(u_in, u_out, levels=None, n=None, nfields=None):
    """Descriptor array for a batch stored as float64 tensors: u_in
    [count, F, M, M, M] on the GPU; u_out either of the same shape (the
    stored layout) or [count, F, n, n, n] (the interior-only layout)."""
    count = int(u_in.shape[0])
    F = int(u_in.shape[1]) if nfields is None else nfields
    M = int(u_in.shape[2])
    n = M - 2 * GHOST if n is None else n
    if tuple(u_out.shape) == tuple(u_in.shape):
        layout, e = OUT_STORED, M
    elif tuple(u_out.shape) == (count, F, n, n, n):
        layout, e = OUT_INTERIOR, n
    else:
        raise ValueError("u_out must have the shape of u_in or [count, F, n, n, n]")
    if not (u_in.is_contiguous() and u_out.is_contiguous()):
        raise ValueError("tensors must be contiguous")
    stride_in = F * M * M * M * 8
    stride_out = F * e * e * e * 8
    arr = (hydro_subgrid_t * max(count, 1))()
    b_in, b_out = _ptr(u_in), _ptr(u_out)
    for s in range(count):
        arr[s].u_in = b_in + s * stride_in
        arr[s].u_out = b_out + s * stride_out
        arr[s].n = n
        arr[s].nfields = F
        arr[s].level = 0 if levels is None else int(levels[s])
        arr[s].out_layout = layout
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


def hydro_step_static(descs, dt: float, dx: float, amax=None, stream=None) -> None:
    """hydro_step through the library's static descriptor table (allocates
    nothing; at most STATIC_MAX sub-grids; overlapping calls on one GPU race)."""
    arr, count = descs
    _check(lib().hydro_step_static(arr, count, float(dt), float(dx), _ptr(amax), _stream(stream)))


def hydro_step26(descs, dt: float, dx: float, amax=None, stream=None) -> None:
    """The 26-point form (9 flux points per face, Simpson's rule), n = 8."""
    arr, count = descs
    _check(lib().hydro_step26(arr, count, float(dt), float(dx), _ptr(amax), _stream(stream)))


def hydro_step_streams(descs, dt: float, dx: float, amax=None, n_streams: int = 1,
                       stream=None) -> None:
    """Strategy 2: one launch per sub-grid over n_streams pool streams."""
    arr, count = descs
    _check(lib().hydro_step_streams(arr, count, float(dt), float(dx), _ptr(amax), int(n_streams),
                                    _stream(stream)))


def hydro_step_each(descs, dt: float, dx: float, amax=None, stream=None) -> None:
    """Baseline: one launch per sub-grid (same kernel)."""
    arr, count = descs
    _check(lib().hydro_step_each(arr, count, float(dt), float(dx), _ptr(amax), _stream(stream)))


def math_check(x, recip_out, rsqrt_out, stream=None) -> None:
    """The kernels' reciprocal and reciprocal square root on device arrays
    (diagnostic)."""
    _check(lib().hydro_math_check(_ptr(x), int(x.numel()), _ptr(recip_out), _ptr(rsqrt_out),
                                  _stream(stream)))


def brick(n, nfields, nb, bc, level=0) -> hydro_brick_t:
    """A brick descriptor: nb = (sub-grids along x, y, z), bc = per-axis
    BC_PERIODIC / BC_OUTFLOW."""
    b = hydro_brick_t()
    b.n, b.nfields, b.level = int(n), int(nfields), int(level)
    for d in range(3):
        b.nb[d] = int(nb[d])
        b.bc[d] = int(bc[d])
    return b


def ghost_fill(b: hydro_brick_t, u, stream=None) -> None:
    """Fill every ghost cell of the brick buffer u (in place)."""
    _check(lib().hydro_ghost_fill(ctypes.byref(b), _ptr(u), _stream(stream)))


def ghost_fill_faces(b: hydro_brick_t, u, stream=None) -> None:
    """Fill the face ghosts of the brick buffer u (in place); edge and corner
    ghosts are left unchanged."""
    _check(lib().hydro_ghost_fill_faces(ctypes.byref(b), _ptr(u), _stream(stream)))


class RK3:
    """SSP-RK3 time-step on a device-resident brick (hydro_rk3_*): u holds
    the state, w and s are work buffers, all brick-sized device tensors."""

    def __init__(self, b: hydro_brick_t, u, w, s):
        self._keep = (b, u, w, s)
        h = ctypes.c_void_p()
        _check(lib().hydro_rk3_create(ctypes.byref(h), ctypes.byref(b), _ptr(u), _ptr(w), _ptr(s)))
        self._h = h

    def stage(self, k: int, dt: float, dx: float, amax=None, stream=None) -> None:
        _check(lib().hydro_rk3_stage(self._h, int(k), float(dt), float(dx), _ptr(amax),
                                     _stream(stream)))

    def step(self, dt: float, dx: float, amax=None, stream=None) -> None:
        _check(lib().hydro_rk3_step(self._h, float(dt), float(dx), _ptr(amax), _stream(stream)))

    def graph(self, dt: float, dx: float, amax=None, stream=None) -> None:
        _check(lib().hydro_rk3_launch_graph(self._h, float(dt), float(dx), _ptr(amax),
                                            _stream(stream)))

    def close(self) -> None:
        if self._h:
            h, self._h = self._h, None
            _check(lib().hydro_rk3_destroy(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


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

    def pattern_floor(self, same_lds: bool = True, stream=None) -> None:
        """The step's HBM access pattern without its arithmetic, over this
        plan's batch (a roofline reference; u_out receives no step result)."""
        _check(lib().hydro_plan_pattern_floor(self._h, int(bool(same_lds)), _stream(stream)))

    def close(self) -> None:
        if self._h:
            _check(lib().hydro_plan_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def region_drive(region, descs, dt: float, dx: float, n_threads: int, mode: int,
                 amax=None) -> float:
    """hydro_region_drive: the tasks of `descs` (subgrids()) from n_threads
    host threads, through `region` (DRIVE_REGION) or one hydro_step launch
    each (DRIVE_EACH; region may be None).  amax: a float64 numpy array of
    one value per task, filled in place, or None.  Returns the wall time in
    seconds."""
    arr, count = descs
    secs = ctypes.c_double()
    ap = None
    if amax is not None:
        assert amax.dtype.name == "float64" and amax.size == count and amax.flags["C_CONTIGUOUS"]
        ap = amax.ctypes.data
    _check(lib().hydro_region_drive(region._h if region is not None else None, arr, int(count),
                                    int(n_threads), float(dt), float(dx), int(mode), ap,
                                    ctypes.byref(secs)))
    return secs.value


def region_kernel(which: int) -> int:
    """Address of a library kernel usable inside a region (REGION_*)."""
    k = lib().hydro_region_kernel(int(which))
    if not k:
        raise HydroError(HYDRO_EINVAL, f"no region kernel {which}")
    return k


class Region:
    """An aggregation region (hydro_region_*): tasks (host threads) that
    enter together form a team sharing chunked buffers; uploads, launches and
    downloads run once for the team, when its last member calls them."""

    def __init__(self, max_team: int, n_streams: int = 1, arena_bytes: int = 1 << 20):
        h = ctypes.c_void_p()
        _check(lib().hydro_region_create(ctypes.byref(h), int(max_team), int(n_streams),
                                         int(arena_bytes)))
        self._h = h

    def enter(self) -> hydro_region_task_t:
        t = hydro_region_task_t()
        _check(lib().hydro_region_enter(self._h, ctypes.byref(t)))
        return t

    def alloc(self, task, nbytes: int):
        """(buffer id, host chunk address, device chunk address)."""
        b = ctypes.c_int32()
        hp, dp = ctypes.c_void_p(), ctypes.c_void_p()
        _check(lib().hydro_region_alloc(self._h, ctypes.byref(task), int(nbytes), ctypes.byref(b),
                                        ctypes.byref(hp), ctypes.byref(dp)))
        return b.value, hp.value, dp.value

    def buffer(self, task, b: int):
        """(device base address, stride) of team buffer b."""
        base, stride = ctypes.c_void_p(), ctypes.c_uint64()
        _check(lib().hydro_region_buffer(self._h, ctypes.byref(task), int(b), ctypes.byref(base),
                                         ctypes.byref(stride)))
        return base.value, stride.value

    def upload(self, task, b: int) -> None:
        _check(lib().hydro_region_upload(self._h, ctypes.byref(task), int(b)))

    def download(self, task, b: int) -> None:
        _check(lib().hydro_region_download(self._h, ctypes.byref(task), int(b)))

    def launch(self, task, kernel: int, blocks_per_task: int, threads: int, args, shmem: int = 0):
        """args: ctypes values (c_void_p, c_int32, c_double, ...) in the
        kernel's parameter order."""
        ptrs = (ctypes.c_void_p * max(len(args), 1))(
            *[ctypes.cast(ctypes.pointer(a), ctypes.c_void_p) for a in args])
        _check(lib().hydro_region_launch(self._h, ctypes.byref(task), kernel, int(blocks_per_task),
                                         int(threads), int(shmem), ptrs))

    def wait(self, task) -> None:
        """Until the team's device work is done; downloaded chunks are then
        valid until leave()."""
        _check(lib().hydro_region_wait(self._h, ctypes.byref(task)))

    def drive(self, descs, dt: float, dx: float, n_threads: int, amax=None) -> float:
        """hydro_region_drive through this region: seconds of wall time."""
        return region_drive(self, descs, dt, dx, n_threads, DRIVE_REGION, amax)

    def leave(self, task) -> None:
        _check(lib().hydro_region_leave(self._h, ctypes.byref(task)))

    def stats(self) -> dict:
        s = hydro_region_stats_t()
        _check(lib().hydro_region_stats(self._h, ctypes.byref(s)))
        d = {n: int(getattr(s, n)) for n, _ in s._fields_ if n != "size_hist"}
        d["size_hist"] = [int(x) for x in s.size_hist]
        return d

    def close(self) -> None:
        if self._h:
            h, self._h = self._h, None
            _check(lib().hydro_region_destroy(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Aggregator:
    """Submit/flush aggregation of sub-grid tasks (hydro_agg_*)."""

    def __init__(self, max_width: int, timeout_us: float = 50.0, n_streams: int = 2,
                 hbm_budget_bytes: int = 0, flush_when_idle: bool = True):
        h = ctypes.c_void_p()
        _check(lib().hydro_agg_create(ctypes.byref(h), int(max_width), float(timeout_us),
                                      int(n_streams), int(hbm_budget_bytes), int(bool(flush_when_idle))))
        self._h = h

    def submit(self, desc, dt: float, dx: float) -> int:
        """desc: a hydro_subgrid_t (or a 1-element descriptor array).  Returns
        the ticket; raises HydroError (code HYDRO_EAGAIN when admission is
        refused)."""
        t = ctypes.c_uint64()
        d = desc if isinstance(desc, hydro_subgrid_t) else desc[0]
        _check(lib().hydro_submit(self._h, ctypes.byref(d), float(dt), float(dx), ctypes.byref(t)))
        return int(t.value)

    def try_submit(self, desc, dt: float, dx: float):
        """Like submit, but returns None instead of raising on HYDRO_EAGAIN."""
        t = ctypes.c_uint64()
        d = desc if isinstance(desc, hydro_subgrid_t) else desc[0]
        rc = lib().hydro_submit(self._h, ctypes.byref(d), float(dt), float(dx), ctypes.byref(t))
        if rc == HYDRO_EAGAIN:
            return None
        _check(rc)
        return int(t.value)

    def submit_many(self, descs, dt: float, dx: float, tickets: bool = False):
        """Submit a batch of tasks in order, as single submits would be
        (hydro_submit_many).  Returns the tickets as a numpy array, or None
        for fire-and-forget tasks (tickets=False; use drain())."""
        import numpy as np
        arr, count = descs
        t = np.zeros(max(count, 1), dtype=np.uint64) if tickets else None
        done = ctypes.c_int32()
        _check(lib().hydro_submit_many(self._h, arr, count, float(dt), float(dx),
                                       None if t is None else t.ctypes.data, ctypes.byref(done)))
        return None if t is None else t[:count]

    def drain(self) -> None:
        """Launch what is held and wait for everything in flight."""
        _check(lib().hydro_agg_drain(self._h))

    def flush(self) -> None:
        _check(lib().hydro_flush(self._h))

    def progress(self) -> None:
        _check(lib().hydro_progress(self._h))

    def poll(self, ticket: int):
        """(done, amax) without blocking; amax is None until done."""
        done = ctypes.c_int32()
        am = ctypes.c_double()
        _check(lib().hydro_poll(self._h, int(ticket), ctypes.byref(done), ctypes.byref(am)))
        return (True, am.value) if done.value else (False, None)

    def wait(self, ticket: int) -> float:
        am = ctypes.c_double()
        _check(lib().hydro_wait(self._h, int(ticket), ctypes.byref(am)))
        return am.value

    def stats(self) -> dict:
        s = hydro_agg_stats_t()
        _check(lib().hydro_agg_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    def close(self) -> None:
        if self._h:
            h, self._h = self._h, None
            _check(lib().hydro_agg_destroy(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def serve_run(pool_descs, task_subgrid, arrival_us, *, nfields, dt, dx, slab_arenas,
              max_width=64, timeout_us=50.0, n_streams=2, flush_when_idle=True,
              keep_slabs=False, want_slabs=False, out_layout=OUT_STORED):
    """Run the serving loop (hydro_serve_run).  slab_arenas: three (tensor or
    None, nslabs) pairs for n = 8, 12, 16, slabs in `out_layout`.  Returns
    (latency_us, amax, slabs, stats) as numpy arrays / dict."""
    import numpy as np
    arr, count = pool_descs
    task_subgrid = np.ascontiguousarray(task_subgrid, dtype=np.int32)
    arrival_us = np.ascontiguousarray(arrival_us, dtype=np.float64)
    n = int(task_subgrid.shape[0])
    cfg = hydro_serve_config_t()
    cfg.max_width, cfg.timeout_us, cfg.n_streams = int(max_width), float(timeout_us), int(n_streams)
    cfg.flush_when_idle, cfg.nfields = int(bool(flush_when_idle)), int(nfields)
    cfg.dt, cfg.dx, cfg.keep_slabs = float(dt), float(dx), int(bool(keep_slabs))
    cfg.out_layout = int(out_layout)
    for e, (t, k) in enumerate(slab_arenas):
        cfg.slab_base[e] = _ptr(t) if t is not None else 0
        cfg.slabs[e] = int(k)
    lat = np.zeros(n, dtype=np.float64)
    am = np.zeros(n, dtype=np.float64)
    slabs = np.zeros(n, dtype=np.uint64) if want_slabs else None
    st = hydro_serve_stats_t()
    _check(lib().hydro_serve_run(ctypes.byref(cfg), arr, count, task_subgrid.ctypes.data,
                                 arrival_us.ctypes.data, n, lat.ctypes.data, am.ctypes.data,
                                 slabs.ctypes.data if want_slabs else None, ctypes.byref(st)))
    stats = {"agg": st.agg.as_dict(), "makespan_us": st.makespan_us,
             "first_admit_us": st.first_admit_us, "max_live": int(st.max_live),
             "slab_waits": int(st.slab_waits), "launch_host_us": st.launch_host_us}
    return lat, am, slabs, stats
