"""Thin Python binding of the C ABI in ``include/sl.h``.

Argument marshalling only: every step of the method runs in the HIP kernels of
``libsl.so``.  PyTorch supplies device memory and streams.  Importing this
module on a machine without the built library raises immediately; there is no
fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsl.so")

SL_OK, SL_EINVAL, SL_ENOMEM, SL_EHIP, SL_ESEARCH, SL_ENEWTON, SL_ENONFINITE, \
    SL_EBUSY, SL_ESTATE, SL_ENOTFOUND, SL_ETOOBIG = 0, -1, -2, -3, -4, -5, -6, -7, -8, -9, -10
SL_STATIC_SCRATCH_BYTES = 128 << 20
SL_STATIC_COUNTERS = 8
SL_FP64, SL_FP32 = 0, 1
SL_RK4, SL_RK3_WILLIAMSON = 0, 1
SL_SRC_NONE, SL_SRC_SHALLOW_WATER = 0, 1
SL_LIMITER_AUTO, SL_LIMITER_IN_TILES, SL_LIMITER_ORDER_WORDS = 0, 1, 2
SL_SERVE_BATCHED, SL_SERVE_QUEUED = 0, 1
SL_MAX_FIELDS = 8
SL_MAX_MODES = 32


class SlVelocity(C.Structure):
    _fields_ = [("kind", C.c_int), ("p", C.c_double * 8), ("nmodes", C.c_int),
                ("modes", C.POINTER(C.c_double))]


class SlGridDesc(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("n", C.c_int64 * 3), ("length", C.c_double * 3),
        ("nfields", C.c_int), ("value_prec", C.c_int), ("order_max", C.c_int),
        ("limiter", C.c_int), ("limiter_theta", C.c_double), ("integrator", C.c_int),
        ("reconstruct_every", C.c_int), ("vel", SlVelocity),
        ("newton_max_iter", C.c_int), ("newton_tol", C.c_double),
        ("walk_max", C.c_int), ("scan_radius", C.c_int), ("eps_inside", C.c_double),
        ("source", C.c_int), ("source_p", C.c_double * 4),
        ("offset", C.c_int64 * 3), ("limiter_pass", C.c_int),
    ]


class SlStats(C.Structure):
    _fields_ = [
        ("nodes", C.c_int64), ("search_fail", C.c_int64), ("newton_fail", C.c_int64),
        ("nonfinite", C.c_int64), ("order_hist", C.c_int64 * 3), ("walked", C.c_int64),
        ("scanned", C.c_int64), ("steps", C.c_int64), ("reconstructs", C.c_int64),
    ]

    def as_dict(self) -> dict:
        return {"nodes": self.nodes, "search_fail": self.search_fail,
                "newton_fail": self.newton_fail, "nonfinite": self.nonfinite,
                "order_hist": list(self.order_hist), "walked": self.walked,
                "scanned": self.scanned, "steps": self.steps,
                "reconstructs": self.reconstructs}


class SlProfile(C.Structure):
    _fields_ = [("traj_launches", C.c_int64), ("traj_ms", C.c_double),
                ("recon_launches", C.c_int64), ("recon_ms", C.c_double),
                ("orders_launches", C.c_int64), ("orders_ms", C.c_double),
                ("source_launches", C.c_int64), ("source_ms", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class SlServerStatus(C.Structure):
    _fields_ = [("active", C.c_int), ("finished", C.c_int), ("bytes_in_use", C.c_size_t),
                ("bytes_free", C.c_size_t), ("ticks", C.c_int64),
                ("completed_ticks", C.c_int64)]


# Every symbol include/sl.h declares, with its ctypes signature.
_VP = C.c_void_p
SIGNATURES = {
    "sl_grid_desc_init": (None, [C.POINTER(SlGridDesc)]),
    "sl_create_grid": (C.c_int, [C.POINTER(SlGridDesc), C.POINTER(_VP)]),
    "sl_destroy_grid": (C.c_int, [_VP]),
    "sl_workspace_bytes": (C.c_size_t, [_VP]),
    "sl_set_velocity_field": (C.c_int, [_VP, C.POINTER(C.POINTER(C.c_double))]),
    "sl_step": (C.c_int, [_VP, _VP, C.c_double, C.c_double, _VP]),
    "sl_reconstruct": (C.c_int, [_VP, _VP, C.POINTER(_VP), C.POINTER(_VP), _VP]),
    "sl_sync": (C.c_int, [_VP, _VP, _VP, C.POINTER(SlStats)]),
    "sl_advance": (C.c_int, [_VP, _VP, C.POINTER(_VP), C.POINTER(_VP), C.c_double,
                             C.c_double, C.c_int, _VP, C.POINTER(C.c_int)]),
    "sl_advance_static": (C.c_int, [_VP, C.POINTER(_VP), C.POINTER(_VP), C.c_double,
                                    C.c_double, C.c_int, _VP, C.POINTER(C.c_int),
                                    C.POINTER(C.c_int64)]),
    "sl_profile_enable": (C.c_int, [_VP, C.c_int]),
    "sl_profile_read": (C.c_int, [_VP, C.POINTER(SlProfile)]),
    "sl_displacement": (C.c_void_p, [_VP, _VP, C.c_int]),
    "sl_strerror": (C.c_char_p, [C.c_int]),
    "sl_version": (C.c_int, []),
    "sl_server_request_bytes": (C.c_size_t, [C.POINTER(SlGridDesc)]),
    "sl_server_arena_overhead": (C.c_size_t, [C.c_int]),
    "sl_server_create": (C.c_int, [_VP, C.c_size_t, C.c_int, C.c_int, _VP, C.POINTER(_VP)]),
    "sl_server_destroy": (C.c_int, [_VP]),
    "sl_server_admit": (C.c_int, [_VP, C.POINTER(SlGridDesc), C.POINTER(_VP), C.c_double,
                                  C.c_double, C.c_int, C.POINTER(C.c_int64)]),
    "sl_server_tick": (C.c_int, [_VP, C.POINTER(C.c_int)]),
    "sl_server_poll": (C.c_int, [_VP, C.POINTER(C.c_int64), C.c_int, C.POINTER(C.c_int)]),
    "sl_server_fetch": (C.c_int, [_VP, C.c_int64, C.POINTER(_VP)]),
    "sl_server_sync": (C.c_int, [_VP, C.POINTER(SlStats)]),
    "sl_server_info": (C.c_int, [_VP, C.POINTER(SlServerStatus)]),
    "sl_server_set_mode": (C.c_int, [_VP, C.c_int, C.c_int]),
    "sl_error_detail": (C.c_char_p, []),
}

_lib = None


def load():
    """Load libsl.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        # PyTorch ships its own HIP runtime (same soname as ROCm's).  Import it
        # first so that libsl.so binds to that runtime instead of loading a
        # second one into the process.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                "libsl.so is not built (%s); run python -m paper_1410_2817_amd.build" % LIB_PATH)
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class SlError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        msg = load().sl_strerror(code).decode()
        if code == SL_EHIP:
            msg += " [%s]" % load().sl_error_detail().decode()
        super().__init__("%s: %s (%d)" % (what, msg, code) if what else "%s (%d)" % (msg, code))


def check(code: int, what: str = "") -> int:
    if code != SL_OK:
        raise SlError(code, what)
    return code


def _stream_handle(stream) -> int | None:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def make_desc(shape: Sequence[int], nfields: int, *, length=None, value_prec="f64",
              order_max=2, limiter=False, theta=0.25, integrator=SL_RK4,
              reconstruct_every=1, vel_kind=0, vel_params=None, modes=None,
              newton_max_iter=20, newton_tol=1e-14, walk_max=32, scan_radius=4,
              eps_inside=1e-12, source=SL_SRC_NONE, source_p=None, offset=None,
              limiter_pass=SL_LIMITER_AUTO):
    """Descriptor for a grid whose arrays have `shape` (array order, x last)."""
    d = SlGridDesc()
    load().sl_grid_desc_init(C.byref(d))
    dim = len(shape)
    d.dim = dim
    length = list(length) if length is not None else [1.0] * dim
    for a in range(dim):  # C side: axis 0 is x
        d.n[a] = int(shape[dim - 1 - a])
        d.length[a] = float(length[dim - 1 - a])
    d.nfields = int(nfields)
    d.value_prec = SL_FP32 if value_prec in ("f32", SL_FP32) else SL_FP64
    d.order_max = int(order_max)
    d.limiter = int(bool(limiter))
    d.limiter_theta = float(theta)
    d.integrator = int(integrator)
    d.reconstruct_every = int(reconstruct_every)
    d.vel.kind = int(vel_kind)
    vp = list(vel_params or []) + [0.0] * 8
    for i in range(8):
        d.vel.p[i] = float(vp[i])
    keep = None
    if modes is not None and len(modes):
        keep = np.ascontiguousarray(modes, dtype=np.float64).reshape(-1, 7)
        d.vel.nmodes = keep.shape[0]
        d.vel.modes = keep.ctypes.data_as(C.POINTER(C.c_double))
    d.newton_max_iter = int(newton_max_iter)
    d.newton_tol = float(newton_tol)
    d.walk_max = int(walk_max)
    d.scan_radius = int(scan_radius)
    d.eps_inside = float(eps_inside)
    if offset is not None:  # array order, like shape
        for a in range(dim):
            d.offset[a] = int(offset[dim - 1 - a])
    d.limiter_pass = int(limiter_pass)
    d.source = int(source)
    sp = list(source_p or []) + [0.0] * 4
    for i in range(4):
        d.source_p[i] = float(sp[i])
    return d, keep


class Grid:
    """A grid handle plus its device workspace (a torch uint8 tensor)."""

    def __init__(self, shape: Sequence[int], nfields: int, device="cuda", **kw):
        import torch
        self.shape = tuple(int(s) for s in shape)
        self.nfields = int(nfields)
        self.value_prec = kw.get("value_prec", "f64")
        self.dtype = torch.float32 if self.value_prec in ("f32", SL_FP32) else torch.float64
        desc, keep = make_desc(shape, nfields, **kw)
        h = _VP()
        check(load().sl_create_grid(C.byref(desc), C.byref(h)), "sl_create_grid")
        del keep  # the library copied the modes
        self._h = h
        self.device = torch.device(device)
        nbytes = int(load().sl_workspace_bytes(h))
        self.workspace = torch.zeros(nbytes, dtype=torch.uint8, device=self.device)
        if self.workspace.data_ptr() % 256:
            raise RuntimeError("workspace is not 256-byte aligned")

    @classmethod
    def from_workload(cls, wl, device="cuda", **over):
        kw = dict(length=wl.length, value_prec=wl.value_prec, order_max=wl.order_max,
                  limiter=wl.limiter, theta=wl.theta, integrator=wl.integrator,
                  reconstruct_every=wl.reconstruct_every, vel_kind=wl.velocity.kind,
                  vel_params=wl.velocity.padded_params(), modes=wl.velocity.modes,
                  source=getattr(wl, "source", SL_SRC_NONE),
                  source_p=list(getattr(wl, "sp", (0.0,) * 4)))
        kw.update(over)
        g = cls(wl.shape, wl.nfields, device=device, **kw)
        if getattr(wl, "ugrid", None) is not None and kw["vel_kind"] == 5:
            g.set_velocity_field(wl.ugrid)
        return g

    def set_velocity_field(self, components):
        """Gridded velocity: copy the samples (components x-first, each of the
        grid's shape) to the device and hand them to the library."""
        import torch
        self._ugrid = [torch.as_tensor(np.asarray(u, dtype=np.float64), device=self.device)
                       .contiguous() for u in components]
        ptrs = (C.POINTER(C.c_double) * len(self._ugrid))(
            *[C.cast(C.c_void_p(u.data_ptr()), C.POINTER(C.c_double)) for u in self._ugrid])
        check(load().sl_set_velocity_field(self._h, ptrs), "sl_set_velocity_field")

    @property
    def nodes(self) -> int:
        return int(np.prod(self.shape))

    def close(self):
        if getattr(self, "_h", None):
            load().sl_destroy_grid(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def new_fields(self, arrays=None):
        import torch
        if arrays is None:
            return [torch.empty(self.shape, dtype=self.dtype, device=self.device)
                    for _ in range(self.nfields)]
        return [torch.as_tensor(np.asarray(a), device=self.device).to(self.dtype).contiguous()
                for a in arrays]

    def _check_fields(self, fs):
        if len(fs) != self.nfields:
            raise ValueError("expected %d fields" % self.nfields)
        for f in fs:
            if tuple(f.shape) != self.shape or f.dtype != self.dtype or not f.is_contiguous() \
                    or f.device != self.device and f.device.type != self.device.type:
                raise ValueError("field must be a contiguous %s tensor of shape %s on %s"
                                 % (self.dtype, self.shape, self.device))

    def step(self, t: float, dt: float, stream=None):
        check(load().sl_step(self._h, C.c_void_p(self.workspace.data_ptr()), float(t),
                             float(dt), C.c_void_p(_stream_handle(stream))), "sl_step")

    def reconstruct(self, fields_in, fields_out, stream=None):
        self._check_fields(fields_in)
        self._check_fields(fields_out)
        fin = (_VP * self.nfields)(*[f.data_ptr() for f in fields_in])
        fout = (_VP * self.nfields)(*[f.data_ptr() for f in fields_out])
        check(load().sl_reconstruct(self._h, C.c_void_p(self.workspace.data_ptr()), fin,
                                    fout, C.c_void_p(_stream_handle(stream))),
              "sl_reconstruct")

    def sync(self, stream=None):
        """Wait, then return (status, stats dict) and clear the counters."""
        st = SlStats()
        rc = load().sl_sync(self._h, C.c_void_p(self.workspace.data_ptr()),
                            C.c_void_p(_stream_handle(stream)), C.byref(st))
        return rc, st.as_dict()

    def displacement(self):
        """The lattice displacement (cell units) as a (dim, *shape) float64 view
        of the workspace, component 0 along x."""
        import torch
        dim = len(self.shape)
        ptr = load().sl_displacement(self._h, C.c_void_p(self.workspace.data_ptr()), 0)
        off = ptr - self.workspace.data_ptr()
        nbytes = 8 * dim * self.nodes
        return self.workspace[off:off + nbytes].view(torch.float64).view(dim, *self.shape)

    def profile(self, period=1):
        """Time every `period`-th launch of each kind (True: every launch;
        False or 0: off)."""
        check(load().sl_profile_enable(self._h, int(period)), "sl_profile_enable")

    def profile_read(self) -> dict:
        p = SlProfile()
        check(load().sl_profile_read(self._h, C.byref(p)), "sl_profile_read")
        return p.as_dict()

    def advance(self, fields, t0: float, dt: float, nsteps: int, out=None, stream=None):
        """nsteps steps from t0 (one sl_advance call; the lattice is reset every
        reconstruct_every steps); returns the set of buffers holding the result,
        which is either `fields` or `out` (allocated when not given)."""
        a = list(fields)
        b = list(out) if out is not None else self.new_fields()
        self._check_fields(a)
        self._check_fields(b)
        pa = (_VP * self.nfields)(*[f.data_ptr() for f in a])
        pb = (_VP * self.nfields)(*[f.data_ptr() for f in b])
        in_b = C.c_int(0)
        check(load().sl_advance(self._h, C.c_void_p(self.workspace.data_ptr()), pa, pb,
                                float(t0), float(dt), int(nsteps),
                                C.c_void_p(_stream_handle(stream)), C.byref(in_b)),
              "sl_advance")
        return b if in_b.value else a

    def advance_static(self, fields, t0: float, dt: float, nsteps: int, out=None,
                       counters=None, stream=None):
        """As advance, through sl_advance_static: the library's static scratch
        on the current device stands in for the workspace (no allocation in the
        call).  `counters`, when given, is a device int64 tensor of at least
        SL_STATIC_COUNTERS elements that receives the call's counters.  Raises
        SlError (SL_ETOOBIG for grids whose workspace exceeds the scratch)."""
        a = list(fields)
        b = list(out) if out is not None else self.new_fields()
        self._check_fields(a)
        self._check_fields(b)
        pa = (_VP * self.nfields)(*[f.data_ptr() for f in a])
        pb = (_VP * self.nfields)(*[f.data_ptr() for f in b])
        in_b = C.c_int(0)
        cp = None
        if counters is not None:
            if counters.numel() < SL_STATIC_COUNTERS or counters.element_size() != 8:
                raise ValueError("counters must hold %d int64 values" % SL_STATIC_COUNTERS)
            cp = C.cast(C.c_void_p(counters.data_ptr()), C.POINTER(C.c_int64))
        check(load().sl_advance_static(self._h, pa, pb, float(t0), float(dt), int(nsteps),
                                       C.c_void_p(_stream_handle(stream)), C.byref(in_b), cp),
              "sl_advance_static")
        return b if in_b.value else a
