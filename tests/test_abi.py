"""The C-ABI library loads, exports every symbol include/sl.h declares, and
validates descriptors on the host (no GPU needed: sl_create_grid does no
device work)."""
import ctypes as C
import os
import re

import pytest

from paper_1410_2817_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "sl.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set()
    for m in re.finditer(r"\b([a-z_][a-z0-9_]*)\s*\(([^;{]*)\)\s*;", text):
        if m.group(1).startswith("sl_"):
            names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        pytest.fail("libsl.so is not built; run python -m paper_1410_2817_amd.build")
    return B.load()


def test_exports_every_declared_symbol(lib):
    names = _declared_functions()
    assert {"sl_create_grid", "sl_step", "sl_reconstruct", "sl_sync"} <= names
    for n in names:
        assert hasattr(lib, n), n
    assert set(B.SIGNATURES) == names
    assert lib.sl_version() == 100


def _desc(**kw):
    d, keep = B.make_desc(kw.pop("shape", (32, 32)), kw.pop("nfields", 1), **kw)
    return d, keep


def _create(d):
    h = C.c_void_p()
    rc = B.load().sl_create_grid(C.byref(d), C.byref(h))
    return rc, h


def test_create_and_workspace_size(lib):
    d, _ = _desc(shape=(40, 48), nfields=3, value_prec="f32", limiter=True)
    rc, h = _create(d)
    assert rc == B.SL_OK and h.value
    ws = lib.sl_workspace_bytes(h)
    n = 40 * 48
    # counters + FP64 displacement (2 components) + one flag byte per node
    assert ws >= 2 * 8 * n + n and ws % 256 == 0
    # the displacement follows the counter block (64 copies of 16 counters)
    assert lib.sl_displacement(h, C.c_void_p(1 << 20), 0) == (1 << 20) + 64 * 16 * 8
    assert lib.sl_displacement(h, C.c_void_p(1 << 20), 2) is None
    assert lib.sl_destroy_grid(h) == B.SL_OK
    assert lib.sl_destroy_grid(None) == B.SL_OK
    assert lib.sl_workspace_bytes(None) == 0


@pytest.mark.parametrize("bad", [
    dict(shape=(32,)), dict(dim=4), dict(shape=(5, 32)),
    dict(nfields=0), dict(nfields=9), dict(order_max=3), dict(order_max=-1),
    dict(value_prec=7), dict(integrator=5), dict(reconstruct_every=0),
    dict(vel_kind=9), dict(vel_kind=2, vel_params=[0.0, 1.0]),  # swirl needs T != 0
    dict(vel_kind=3, vel_params=[3.0, 1.0]),  # 3-D family on a 2-D grid
    dict(vel_kind=4),  # Fourier without modes
    dict(newton_max_iter=0), dict(newton_tol=0.0), dict(scan_radius=99),
    dict(length=(1.0, 0.0)), dict(vel_params=[float("nan")]), dict(limiter_pass=3),
    # size limits: 2^30 nodes in all, n_x above 2^24, n_y above 4 x 65535,
    # n_z above 65535 (array order: x last)
    dict(shape=(1024, 1024, 1024)), dict(shape=(8, (1 << 24) + 1)),
    dict(shape=(4 * 65535 + 1, 8)), dict(shape=(65536, 8, 8)),
])
def test_create_rejects_bad_descriptors(lib, bad):
    kw = dict(bad)
    if "dim" in kw:
        d, keep = _desc(shape=(8, 8, 8))
        d.dim = kw["dim"]
    elif kw.get("value_prec") == 7:
        d, keep = _desc()
        d.value_prec = 7
    elif kw.get("vel_kind") == 4:
        d, keep = _desc(vel_kind=4)
        d.vel.nmodes = 0
    else:
        d, keep = _desc(**kw)
    rc, h = _create(d)
    assert rc == B.SL_EINVAL and not h.value


@pytest.mark.parametrize("shape", [(1023, 1024, 1024), (65535, 8, 8), (4 * 65535, 8),
                                   (8, 1 << 24)])
def test_create_accepts_the_largest_grids(lib, shape):
    # The largest grid (2^30 - 2^20 nodes) and each axis at its limit: the
    # workspace holds at least the two FP64 displacement sets.
    d, _ = _desc(shape=shape, limiter=True)
    rc, h = _create(d)
    assert rc == B.SL_OK and h.value
    n = 1
    for s in shape:
        n *= s
    assert lib.sl_workspace_bytes(h) >= 2 * 8 * len(shape) * n
    assert lib.sl_destroy_grid(h) == B.SL_OK


def test_null_arguments(lib):
    assert lib.sl_create_grid(None, None) == B.SL_EINVAL
    h = C.c_void_p()
    assert lib.sl_create_grid(None, C.byref(h)) == B.SL_EINVAL
    d, _ = _desc()
    rc, h = _create(d)
    assert rc == 0
    # Host-side argument checks reject before any device work.
    assert lib.sl_step(None, C.c_void_p(256), 0.0, 0.1, None) == B.SL_EINVAL
    assert lib.sl_step(h, None, 0.0, 0.1, None) == B.SL_EINVAL
    assert lib.sl_step(h, C.c_void_p(257), 0.0, 0.1, None) == B.SL_EINVAL
    assert lib.sl_step(h, C.c_void_p(256), float("nan"), 0.1, None) == B.SL_EINVAL
    arr = (C.c_void_p * 1)(256)
    # reconstruct before any step is out of order
    assert lib.sl_reconstruct(h, C.c_void_p(256), arr, arr, None) == B.SL_ESTATE
    assert lib.sl_reconstruct(h, None, arr, arr, None) == B.SL_EINVAL
    assert lib.sl_sync(None, None, None, None) == B.SL_EINVAL
    lib.sl_destroy_grid(h)


def test_strerror(lib):
    for code in range(0, -10, -1):
        assert lib.sl_strerror(code)
    assert lib.sl_strerror(-1234) == b"unknown status"


def test_fourier_modes_are_copied(lib):
    import numpy as np
    modes = np.array([[1, 2, 0, 0.5, 0, 0, 0.3]], dtype=np.float64)
    d, keep = _desc(vel_kind=4, vel_params=[1.0], modes=modes)
    rc, h = _create(d)
    assert rc == 0
    keep[:] = np.nan  # the library must not read the caller's array later
    lib.sl_destroy_grid(h)


def test_gridded_velocity_state_and_validation(lib):
    """A gridded velocity needs its samples before stepping (checked on the
    host, before any device work); the order must be 0..2; the setter only
    applies to gridded grids and rejects NULL."""
    d, _ = _desc(shape=(16, 16), vel_kind=5, vel_params=[2.0])
    rc, h = _create(d)
    assert rc == B.SL_OK
    ws = C.c_void_p(1 << 20)
    assert lib.sl_step(h, ws, 0.0, 0.1, None) == B.SL_ESTATE
    assert lib.sl_advance(h, ws, None, None, 0.0, 0.1, 0, None, None) in (B.SL_EINVAL, B.SL_ESTATE)
    assert lib.sl_set_velocity_field(h, None) == B.SL_EINVAL
    null2 = (C.POINTER(C.c_double) * 2)()
    assert lib.sl_set_velocity_field(h, null2) == B.SL_EINVAL
    assert lib.sl_destroy_grid(h) == B.SL_OK
    for order in (3.0, 0.5, -1.0):
        d, _ = _desc(shape=(16, 16), vel_kind=5, vel_params=[order])
        rc, h = _create(d)
        assert rc == B.SL_EINVAL
    d, _ = _desc(shape=(16, 16))
    rc, h = _create(d)
    fake = (C.POINTER(C.c_double) * 2)(C.cast(C.c_void_p(4096), C.POINTER(C.c_double)),
                                      C.cast(C.c_void_p(8192), C.POINTER(C.c_double)))
    assert lib.sl_set_velocity_field(h, fake) == B.SL_EINVAL
    assert lib.sl_destroy_grid(h) == B.SL_OK


def test_carried_velocity_validation(lib):
    """A carried velocity needs the velocity components among the fields and
    runs through sl_advance (sl_step has no fields)."""
    d, _ = _desc(shape=(16, 16), nfields=1, vel_kind=6)
    rc, h = _create(d)
    assert rc == B.SL_EINVAL
    d, _ = _desc(shape=(16, 16), nfields=2, vel_kind=6)
    rc, h = _create(d)
    assert rc == B.SL_OK
    assert lib.sl_step(h, C.c_void_p(1 << 20), 0.0, 0.1, None) == B.SL_EINVAL
    assert lib.sl_destroy_grid(h) == B.SL_OK


def test_shallow_water_source_validation(lib):
    """The shallow-water source needs a 2-D grid, a carried velocity, at least
    (u1, u2, h), the low-storage RK3 and a reset every step; its workspace
    holds the lattice values, the stage fields and the RK registers on top of
    the plain grid's."""
    ok = dict(shape=(16, 20), nfields=3, vel_kind=6, integrator=B.SL_RK3_WILLIAMSON,
              source=B.SL_SRC_SHALLOW_WATER, source_p=[0.0, 250.0, 0.5, 0.0])
    d, _ = _desc(**ok)
    rc, h = _create(d)
    assert rc == B.SL_OK
    ws = lib.sl_workspace_bytes(h)
    n = 16 * 20
    d0, _ = _desc(shape=(16, 20), nfields=3, vel_kind=6, integrator=B.SL_RK3_WILLIAMSON)
    rc0, h0 = _create(d0)
    assert rc0 == B.SL_OK
    # + 2 x 3 value planes, 2 + 3 FP64 register planes
    assert ws - lib.sl_workspace_bytes(h0) >= 6 * 8 * n + 5 * 8 * n
    assert lib.sl_step(h, C.c_void_p(1 << 20), 0.0, 0.1, None) == B.SL_EINVAL
    lib.sl_destroy_grid(h0)
    assert lib.sl_destroy_grid(h) == B.SL_OK
    for bad in (dict(nfields=2), dict(vel_kind=0), dict(integrator=B.SL_RK4),
                dict(reconstruct_every=2), dict(shape=(8, 8, 8)),
                dict(source=7), dict(source_p=[0.0, float("inf"), 0.5, 0.0]),
                dict(source_p=[0.0, 1.0, 0.5, -1e-3])):
        kw = dict(ok)
        kw.update(bad)
        d, _ = _desc(**kw)
        rc, h = _create(d)
        assert rc == B.SL_EINVAL and not h.value, bad


def test_server_arena_overhead(lib):
    # The server's own share of the arena grows with its request slots and is
    # 256-byte granular; invalid slot counts give 0.
    a, b = lib.sl_server_arena_overhead(2), lib.sl_server_arena_overhead(256)
    assert 0 < a < b and a % 256 == 0 and b % 256 == 0
    assert lib.sl_server_arena_overhead(0) == 0 and lib.sl_server_arena_overhead(5000) == 0
