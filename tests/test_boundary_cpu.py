"""The C-ABI library loads on the CPU host and exports every symbol that
include/hydroagg.h declares; argument checks answer without touching a GPU."""
import ctypes
import os
import re

import pytest

from paper_2210_06438_amd import hydroagg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(hydro_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    L = hydroagg.lib()
    names = declared_functions()
    assert "hydro_step" in names and "hydro_last_error" in names
    for n in names:
        assert hasattr(L, n), n


def test_descriptor_is_32_bytes():
    assert ctypes.sizeof(hydroagg.hydro_subgrid_t) == 32


STORED_8_11 = 11 * 14 ** 3 * 8      # bytes of an 8^3, F = 11 sub-grid with ghosts
INTERIOR_8_11 = 11 * 8 ** 3 * 8


def _desc(n=8, nf=11, level=0, out_layout=0, u_in=0x100000, u_out=0x10000000):
    a = (hydroagg.hydro_subgrid_t * 1)()
    a[0].u_in, a[0].u_out, a[0].n, a[0].nfields = u_in, u_out, n, nf
    a[0].level, a[0].out_layout = level, out_layout
    return a


@pytest.mark.parametrize("fn", ["hydro_step", "hydro_step_each", "hydro_step_static"])
@pytest.mark.parametrize("kw,count,dt,dx", [
    (dict(n=9), 1, 0.1, 0.1),
    (dict(nf=7), 1, 0.1, 0.1),
    (dict(level=-1), 1, 0.1, 0.1),
    (dict(level=31), 1, 0.1, 0.1),
    (dict(out_layout=2), 1, 0.1, 0.1),
    (dict(out_layout=-1), 1, 0.1, 0.1),
    (dict(u_in=0), 1, 0.1, 0.1),
    (dict(u_out=0x100000), 1, 0.1, 0.1),
    # u_out overlapping u_in by one double, either side, either layout
    (dict(u_out=0x100000 + STORED_8_11 - 8), 1, 0.1, 0.1),
    (dict(u_out=0x100000 - STORED_8_11 + 8), 1, 0.1, 0.1),
    (dict(u_out=0x100000 - INTERIOR_8_11 + 8, out_layout=1), 1, 0.1, 0.1),
    (dict(u_out=0x100008), 1, 0.1, 0.1),
    (dict(), -1, 0.1, 0.1),
    (dict(), 1, -0.1, 0.1),
    (dict(), 1, float("nan"), 0.1),
    (dict(), 1, float("inf"), 0.1),
    (dict(), 1, 0.1, 0.0),
    (dict(), 1, 0.1, float("inf")),
])
def test_bad_arguments_are_rejected_before_any_gpu_call(fn, kw, count, dt, dx):
    L = hydroagg.lib()
    rc = getattr(L, fn)(_desc(**kw), count, dt, dx, None, None)
    assert rc == hydroagg.HYDRO_EINVAL
    assert L.hydro_last_error().decode() != ""


def test_null_batch_and_empty_batch():
    L = hydroagg.lib()
    assert L.hydro_step(None, 1, 0.1, 0.1, None, None) == hydroagg.HYDRO_EINVAL
    assert L.hydro_step(None, 0, 0.1, 0.1, None, None) == hydroagg.HYDRO_OK
    assert L.hydro_step_each(None, 0, 0.1, 0.1, None, None) == hydroagg.HYDRO_OK
    assert L.hydro_step_static(None, 0, 0.1, 0.1, None, None) == hydroagg.HYDRO_OK


def test_static_step_rejects_batches_beyond_its_table():
    """hydro_step_static holds at most STATIC_MAX descriptors; one more is an
    argument error, reported before any device call."""
    L = hydroagg.lib()
    n = hydroagg.STATIC_MAX + 1
    a = (hydroagg.hydro_subgrid_t * n)()
    for i in range(n):
        a[i].u_in, a[i].u_out = 0x100000 + i * 2 * STORED_8_11, 0x100000 + (2 * i + 1) * STORED_8_11
        a[i].n, a[i].nfields = 8, 11
    assert L.hydro_step_static(a, n, 0.1, 0.1, None, None) == hydroagg.HYDRO_EINVAL
    assert "HYDRO_STATIC_MAX" in L.hydro_last_error().decode()


def test_tile_setting_is_validated_and_round_trips():
    L = hydroagg.lib()
    defaults = {(n, f): hydroagg.get_tile(n, f) for n in (8, 12, 16) for f in (6, 11)}
    assert defaults == {(8, 6): 8, (8, 11): 8, (12, 6): 4, (12, 11): 4, (16, 6): 8, (16, 11): 8}
    for args in ((9, 11, 8), (8, 7, 8), (8, 11, 5), (8, 11, 0), (12, 6, 16)):
        assert L.hydro_set_tile(*args) == hydroagg.HYDRO_EINVAL
    assert L.hydro_get_tile(8, 11, None) == hydroagg.HYDRO_EINVAL
    try:
        hydroagg.set_tile(16, 6, 4)
        assert hydroagg.get_tile(16, 6) == 4 and hydroagg.get_tile(16, 11) == 8
    finally:
        hydroagg.set_tile(16, 6, defaults[(16, 6)])
    assert hydroagg.get_tile(16, 6) == 8


def test_math_check_arguments():
    L = hydroagg.lib()
    assert L.hydro_math_check(None, -1, None, None, None) == hydroagg.HYDRO_EINVAL
    assert L.hydro_math_check(None, 4, None, None, None) == hydroagg.HYDRO_EINVAL
    assert L.hydro_math_check(None, 0, None, None, None) == hydroagg.HYDRO_OK


def test_brick_arguments_are_rejected_before_any_gpu_call():
    L = hydroagg.lib()
    good = dict(n=8, nf=6, nb=(2, 2, 2), bc=(0, 0, 0), level=0)
    bad = [dict(n=10), dict(nf=7), dict(nb=(0, 1, 1)), dict(nb=(1, -1, 1)), dict(bc=(0, 2, 0)),
           dict(bc=(-1, 0, 0)), dict(level=31), dict(nb=(1024, 1024, 2))]
    for kw in bad:
        a = {**good, **kw}
        b = hydroagg.brick(a["n"], a["nf"], a["nb"], a["bc"], a["level"])
        assert L.hydro_ghost_fill(ctypes.byref(b), 0x100000, None) == hydroagg.HYDRO_EINVAL, kw
        h = ctypes.c_void_p()
        assert L.hydro_rk3_create(ctypes.byref(h), ctypes.byref(b), 0x100000, 0x20000000,
                                  0x40000000) == hydroagg.HYDRO_EINVAL, kw
    b = hydroagg.brick(8, 6, (2, 2, 2), (0, 0, 0))
    assert L.hydro_ghost_fill(None, 0x100000, None) == hydroagg.HYDRO_EINVAL
    assert L.hydro_ghost_fill(ctypes.byref(b), 0, None) == hydroagg.HYDRO_EINVAL
    assert L.hydro_ghost_fill(ctypes.byref(b), 0x100008, None) == hydroagg.HYDRO_EINVAL
    h = ctypes.c_void_p()
    size = 8 * 6 * 14 ** 3 * 8
    # overlapping buffers, a NULL buffer, a NULL out pointer
    assert L.hydro_rk3_create(ctypes.byref(h), ctypes.byref(b), 0x100000, 0x100000 + size - 8,
                              0x40000000) == hydroagg.HYDRO_EINVAL
    assert L.hydro_rk3_create(ctypes.byref(h), ctypes.byref(b), 0x100000, 0,
                              0x40000000) == hydroagg.HYDRO_EINVAL
    assert L.hydro_rk3_create(None, ctypes.byref(b), 0x100000, 0x20000000,
                              0x40000000) == hydroagg.HYDRO_EINVAL
    for fn in (L.hydro_rk3_step, L.hydro_rk3_launch_graph):
        assert fn(None, 0.1, 0.1, None, None) == hydroagg.HYDRO_EINVAL
    assert L.hydro_rk3_stage(None, 1, 0.1, 0.1, None, None) == hydroagg.HYDRO_EINVAL
    assert L.hydro_rk3_destroy(None) == hydroagg.HYDRO_OK


def test_pattern_floor_needs_a_plan():
    L = hydroagg.lib()
    assert L.hydro_plan_pattern_floor(None, 1, None) == hydroagg.HYDRO_EINVAL


def test_strategy_and_bulk_calls_check_arguments():
    L = hydroagg.lib()
    for k in (0, -1, 129):
        assert L.hydro_step_streams(_desc(), 1, 0.1, 0.1, None, k, None) == hydroagg.HYDRO_EINVAL
    assert L.hydro_step_streams(_desc(n=9), 1, 0.1, 0.1, None, 4, None) == hydroagg.HYDRO_EINVAL
    n = ctypes.c_int32()
    assert L.hydro_submit_many(None, _desc(), 1, 0.1, 0.1, None, ctypes.byref(n)) == \
        hydroagg.HYDRO_EINVAL
    assert L.hydro_agg_drain(None) == hydroagg.HYDRO_EINVAL
    h = ctypes.c_void_p()
    for k in (0, 129):
        assert L.hydro_agg_create(ctypes.byref(h), 4, 50.0, k, 0, 1) == hydroagg.HYDRO_EINVAL


def test_region_calls_check_arguments():
    L = hydroagg.lib()
    h = ctypes.c_void_p()
    for args in ((0, 1, 1 << 20), (4, 0, 1 << 20), (4, 33, 1 << 20), (4, 1, 16)):
        assert L.hydro_region_create(ctypes.byref(h), *args) == hydroagg.HYDRO_EINVAL, args
    assert L.hydro_region_create(None, 4, 1, 1 << 20) == hydroagg.HYDRO_EINVAL
    t = hydroagg.hydro_region_task_t()
    assert L.hydro_region_enter(None, ctypes.byref(t)) == hydroagg.HYDRO_EINVAL
    assert L.hydro_region_leave(None, ctypes.byref(t)) == hydroagg.HYDRO_EINVAL
    assert L.hydro_region_destroy(None) == hydroagg.HYDRO_OK
    for k in (hydroagg.REGION_STEP8_F6, hydroagg.REGION_STEP8_F11, hydroagg.REGION_AXPBY):
        assert L.hydro_region_kernel(k)
    assert not L.hydro_region_kernel(3)
    assert ctypes.sizeof(hydroagg.hydro_region_task_t) == 24
    assert ctypes.sizeof(hydroagg.hydro_region_axpby_t) == 48
