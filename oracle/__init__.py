"""ctypes binding of the plain FP64 CPU oracle (``sl_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg of
the benchmark use this module to check the GPU library; the GPU library never
imports it and shares no code with it.

Arrays follow the mesh layout of the paper's regular reference grid (Sec. 2.1):
a field of an ``(nz, ny, nx)`` grid is a C-ordered array with x fastest, and a
displacement array has shape ``(dim, *grid)`` with component 0 along x, in
cell units.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sl_oracle.c")
_LIB = os.path.join(_HERE, "libsl_oracle.so")

OK, EINVAL, ESEARCH, ENEWTON = 0, -1, -4, -5
RK4, RK3_WILLIAMSON = 0, 1
VEL_UNIFORM, VEL_SOLID_BODY, VEL_SWIRL2D, VEL_DEFORM3D, VEL_FOURIER, VEL_GRIDDED, VEL_CARRIED = range(7)
SRC_NONE, SRC_SHALLOW_WATER = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-std=gnu11", "-O2", "-fopenmp", "-fPIC", "-shared",
             "-ffp-contract=off", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("nfields", C.c_int),
        ("n", C.c_int64 * 3), ("len", C.c_double * 3),
        ("order_max", C.c_int), ("limiter", C.c_int), ("theta", C.c_double),
        ("integrator", C.c_int), ("vel_kind", C.c_int), ("vp", C.c_double * 8),
        ("nmodes", C.c_int), ("modes", C.POINTER(C.c_double)),
        ("newton_max_iter", C.c_int), ("newton_tol", C.c_double),
        ("walk_max", C.c_int), ("eps_inside", C.c_double),
        ("scan_radius", C.c_int),
        ("ugrid", C.POINTER(C.c_double) * 3),
        ("src_kind", C.c_int), ("sp", C.c_double * 4),
        ("offset", C.c_int64 * 3),
    ]


class _Stats(C.Structure):
    _fields_ = [
        ("nodes", C.c_int64), ("search_fail", C.c_int64), ("newton_fail", C.c_int64),
        ("order_hist", C.c_int64 * 3), ("flagged", C.c_int64),
        ("walk_steps", C.c_int64), ("newton_iters", C.c_int64),
    ]

    def as_dict(self) -> dict:
        return {
            "nodes": self.nodes, "search_fail": self.search_fail,
            "newton_fail": self.newton_fail, "order_hist": list(self.order_hist),
            "flagged": self.flagged, "walk_steps": self.walk_steps,
            "newton_iters": self.newton_iters,
        }


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = C.CDLL(_LIB)
        P = C.POINTER(_Problem)
        dp = C.POINTER(C.c_double)
        i64p = C.POINTER(C.c_int64)
        lib.orc_zspline.argtypes = [C.c_int, C.c_double]
        lib.orc_zspline.restype = C.c_double
        lib.orc_weights.argtypes = [C.c_int, C.c_double, dp]
        lib.orc_velocity.argtypes = [P, dp, C.c_double, dp]
        lib.orc_trajectory.argtypes = [P, i64p, C.c_double, C.c_double, dp]
        lib.orc_trajectories.argtypes = [P, C.c_double, C.c_double, dp]
        lib.orc_flag.argtypes = [P, dp, i64p]
        lib.orc_flag.restype = C.c_int
        lib.orc_flags.argtypes = [P, C.POINTER(dp), C.POINTER(C.c_uint8)]
        lib.orc_locate.argtypes = [P, dp, i64p, i64p, dp, C.POINTER(C.c_int),
                                   C.POINTER(C.c_int)]
        lib.orc_locate.restype = C.c_int
        lib.orc_reconstruct.argtypes = [P, dp, C.POINTER(dp), C.POINTER(dp),
                                        C.POINTER(_Stats), C.POINTER(C.c_int8)]
        lib.orc_reconstruct.restype = C.c_int
        lib.orc_step_sampled.argtypes = [P, C.c_double, C.c_double, C.c_int,
                                         C.POINTER(dp), i64p, C.c_int64, dp,
                                         C.POINTER(_Stats)]
        lib.orc_step_sampled.restype = C.c_int
        lib.orc_run.argtypes = [P, C.c_double, C.c_double, C.c_int, C.c_int,
                                C.POINTER(dp), C.POINTER(_Stats)]
        lib.orc_run.restype = C.c_int
        lib.orc_run_f32store.argtypes = lib.orc_run.argtypes
        lib.orc_run_f32store.restype = C.c_int
        lib.orc_fd_weights.argtypes = [C.c_int, C.c_int, dp]
        lib.orc_fd_weights.restype = C.c_int
        lib.orc_source_mesh.argtypes = [P, C.POINTER(dp), C.POINTER(dp)]
        lib.orc_source_mesh.restype = C.c_int
        lib.orc_run_source.argtypes = [P, C.c_double, C.c_double, C.c_int,
                                       C.POINTER(dp), C.POINTER(_Stats)]
        lib.orc_run_source.restype = C.c_int
        lib.orc_threads.argtypes = []
        lib.orc_threads.restype = C.c_int
        _lib = lib
    return _lib


@dataclass
class Problem:
    """One advection problem on a periodic node-centred grid.

    ``shape`` is the grid in array order (slowest axis first, x last), the
    same order the field arrays use; ``length`` is the physical extent per
    array axis.  Velocity kinds and their parameters are described in
    ``sl_oracle.c`` (``orc_velocity``)."""

    shape: Sequence[int]
    nfields: int = 1
    length: Sequence[float] | None = None
    order_max: int = 2
    limiter: bool = False
    theta: float = 0.25
    integrator: int = RK4
    vel_kind: int = VEL_UNIFORM
    vp: Sequence[float] = field(default_factory=lambda: [0.0] * 8)
    modes: np.ndarray | None = None
    newton_max_iter: int = 20
    newton_tol: float = 1e-14
    walk_max: int = 32
    eps_inside: float = 1e-12
    scan_radius: int = 4
    # VEL_GRIDDED: velocity components on the mesh nodes, each of `shape`
    # (array order), listed x-first; vp[0] is the interpolation order.
    ugrid: Sequence[np.ndarray] | None = None
    # Source term (orc_source_mesh): SRC_SHALLOW_WATER with sp = (fc, beta,
    # y0, nu); fields are u1, u2, h (x-first velocity), then passive ones.
    src_kind: int = SRC_NONE
    sp: Sequence[float] = field(default_factory=lambda: [0.0] * 4)
    # Index of node 0 in a larger lattice (array order, like shape).
    offset: Sequence[int] | None = None

    @property
    def dim(self) -> int:
        return len(self.shape)

    def _c(self) -> _Problem:
        p = _Problem()
        p.dim = self.dim
        p.nfields = self.nfields
        ln = list(self.length) if self.length is not None else [1.0] * self.dim
        # The C side indexes axes x-first.
        for a in range(self.dim):
            p.n[a] = int(self.shape[self.dim - 1 - a])
            p.len[a] = float(ln[self.dim - 1 - a])
        p.order_max = self.order_max
        p.limiter = int(bool(self.limiter))
        p.theta = self.theta
        p.integrator = self.integrator
        p.vel_kind = self.vel_kind
        vp = list(self.vp) + [0.0] * (8 - len(self.vp))
        for i in range(8):
            p.vp[i] = float(vp[i])
        if self.modes is not None and len(self.modes):
            m = np.ascontiguousarray(self.modes, dtype=np.float64).reshape(-1, 7)
            self._modes_keep = m
            p.nmodes = m.shape[0]
            p.modes = m.ctypes.data_as(C.POINTER(C.c_double))
        else:
            p.nmodes = 0
            p.modes = None
        p.newton_max_iter = self.newton_max_iter
        p.newton_tol = self.newton_tol
        p.walk_max = self.walk_max
        p.eps_inside = self.eps_inside
        p.scan_radius = self.scan_radius
        if self.offset is not None:
            for a in range(self.dim):
                p.offset[a] = int(self.offset[self.dim - 1 - a])
        p.src_kind = int(self.src_kind)
        spv = list(self.sp) + [0.0] * (4 - len(self.sp))
        for i in range(4):
            p.sp[i] = float(spv[i])
        if self.ugrid is not None:
            keep = [np.ascontiguousarray(u, dtype=np.float64) for u in self.ugrid]
            self._ugrid_keep = keep
            for a, u in enumerate(keep):
                p.ugrid[a] = u.ctypes.data_as(C.POINTER(C.c_double))
        return p


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _fields_ptrs(fields: Sequence[np.ndarray]):
    arr = (C.POINTER(C.c_double) * len(fields))()
    for i, f in enumerate(fields):
        arr[i] = _dp(f)
    return arr


def _as_fields(prob: Problem, fields) -> list[np.ndarray]:
    fs = [np.ascontiguousarray(f, dtype=np.float64) for f in fields]
    assert len(fs) == prob.nfields
    for f in fs:
        assert tuple(f.shape) == tuple(prob.shape), (f.shape, prob.shape)
    return fs


def zspline(m: int, x: float) -> float:
    """Cardinal Z-spline basis function of order m at x (Appendix)."""
    return _load().orc_zspline(m, float(x))


def weights(m: int, t: float) -> np.ndarray:
    """Weights Z_m(t - k), k = -m..m+1, of the nodes around a point r + t."""
    w = np.zeros(2 * m + 2)
    _load().orc_weights(m, float(t), _dp(w))
    return w


def velocity(prob: Problem, x: Sequence[float], t: float) -> np.ndarray:
    """Velocity at a physical point, components x-first."""
    xa = np.zeros(3)
    xa[: prob.dim] = x
    u = np.zeros(3)
    p = prob._c()
    _load().orc_velocity(C.byref(p), _dp(xa), float(t), _dp(u))
    return u[: prob.dim].copy()


def trajectory(prob: Problem, node: Sequence[int], t: float, dt: float,
               disp: Sequence[float] | None = None) -> np.ndarray:
    """Displacement (cell units, x-first) of one lattice node after one step."""
    nd = np.zeros(3, dtype=np.int64)
    nd[: prob.dim] = node
    d = np.zeros(3)
    if disp is not None:
        d[: prob.dim] = disp
    p = prob._c()
    _load().orc_trajectory(C.byref(p), nd.ctypes.data_as(C.POINTER(C.c_int64)),
                           float(t), float(dt), _dp(d))
    return d[: prob.dim].copy()


def trajectories(prob: Problem, t: float, dt: float,
                 disp: np.ndarray | None = None) -> np.ndarray:
    """Displacements of all lattice nodes after one step, shape (dim, *shape)."""
    if disp is None:
        disp = np.zeros((prob.dim, *prob.shape))
    d = np.ascontiguousarray(disp, dtype=np.float64).copy()
    p = prob._c()
    _load().orc_trajectories(C.byref(p), float(t), float(dt), _dp(d))
    return d


def flag(prob: Problem, field_: np.ndarray, node: Sequence[int]) -> int:
    f = np.ascontiguousarray(field_, dtype=np.float64)
    nd = np.zeros(3, dtype=np.int64)
    nd[: prob.dim] = node
    p = prob._c()
    return _load().orc_flag(C.byref(p), _dp(f), nd.ctypes.data_as(C.POINTER(C.c_int64)))


def flags(prob: Problem, fields) -> np.ndarray:
    """Jump flags of all lattice points, bit f set for field f."""
    fs = _as_fields(prob, fields)
    out = np.zeros(prob.shape, dtype=np.uint8)
    p = prob._c()
    _load().orc_flags(C.byref(p), _fields_ptrs(fs), out.ctypes.data_as(C.POINTER(C.c_uint8)))
    return out


def locate(prob: Problem, disp: np.ndarray, target: Sequence[int]):
    """Element search + Newton for one mesh node (x-first integer coords).

    Returns (status, r, xi, walk_steps, newton_iters)."""
    d = np.ascontiguousarray(disp, dtype=np.float64)
    tg = np.zeros(3, dtype=np.int64)
    tg[: prob.dim] = target
    r = np.zeros(3, dtype=np.int64)
    xi = np.zeros(3)
    ws, ni = C.c_int(0), C.c_int(0)
    p = prob._c()
    rc = _load().orc_locate(C.byref(p), _dp(d), tg.ctypes.data_as(C.POINTER(C.c_int64)),
                            r.ctypes.data_as(C.POINTER(C.c_int64)), _dp(xi),
                            C.byref(ws), C.byref(ni))
    return rc, r[: prob.dim].copy(), xi[: prob.dim].copy(), ws.value, ni.value


def reconstruct(prob: Problem, disp: np.ndarray, fields, orders: bool = False):
    """Reconstruct every mesh node from a lattice displacement.

    Returns (status, list of output fields, stats dict), plus the per-field,
    per-node interpolation order (int8, -1 where the search failed) when
    ``orders`` is set."""
    fs = _as_fields(prob, fields)
    d = np.ascontiguousarray(disp, dtype=np.float64)
    assert d.shape == (prob.dim, *prob.shape)
    outs = [np.empty(prob.shape) for _ in range(prob.nfields)]
    st = _Stats()
    p = prob._c()
    om = np.empty((prob.nfields, *prob.shape), dtype=np.int8) if orders else None
    rc = _load().orc_reconstruct(
        C.byref(p), _dp(d), _fields_ptrs(fs), _fields_ptrs(outs), C.byref(st),
        om.ctypes.data_as(C.POINTER(C.c_int8)) if orders else None)
    if orders:
        return rc, outs, st.as_dict(), om
    return rc, outs, st.as_dict()


def step(prob: Problem, t: float, dt: float, fields):
    """One full step (trajectories from a reset lattice, then reconstruction)."""
    disp = trajectories(prob, t, dt)
    return reconstruct(prob, disp, fields)


def step_sampled(prob: Problem, t: float, dt: float, fields, nodes,
                 ksteps: int = 1):
    """One full step evaluated only at the given mesh nodes (flat indices),
    integrating every trajectory the search touches on demand.

    Returns (status, out array of shape (count, nfields), stats dict)."""
    fs = _as_fields(prob, fields)
    idx = np.ascontiguousarray(nodes, dtype=np.int64).ravel()
    out = np.empty((idx.size, prob.nfields))
    st = _Stats()
    p = prob._c()
    rc = _load().orc_step_sampled(C.byref(p), float(t), float(dt), int(ksteps),
                                  _fields_ptrs(fs),
                                  idx.ctypes.data_as(C.POINTER(C.c_int64)),
                                  int(idx.size), _dp(out), C.byref(st))
    return rc, out, st.as_dict()


def run(prob: Problem, t0: float, dt: float, nsteps: int, fields, kevery: int = 1,
        store: str = "f64"):
    """nsteps steps from t0; returns (status, fields, accumulated stats).

    store="f32" rounds the fields to FP32 after every reconstruction (the
    values a run with FP32 field storage carries between steps); the
    arithmetic stays FP64."""
    fs = [f.copy() for f in _as_fields(prob, fields)]
    st = _Stats()
    p = prob._c()
    fn = _load().orc_run_f32store if store == "f32" else _load().orc_run
    rc = fn(C.byref(p), float(t0), float(dt), int(nsteps), int(kevery),
            _fields_ptrs(fs), C.byref(st))
    return rc, fs, st.as_dict()


def fd_weights(half_width: int, deriv: int) -> np.ndarray:
    """Centred finite-difference weights of the given derivative on a unit
    grid, offsets -half_width..half_width."""
    c = np.zeros(2 * half_width + 1)
    rc = _load().orc_fd_weights(int(half_width), int(deriv), _dp(c))
    if rc != OK:
        raise ValueError("orc_fd_weights failed")
    return c


def source_mesh(prob: Problem, fields):
    """Right-hand side of the shallow-water system on the mesh for the given
    fields (u1, u2, h, ...); returns (status, [S_u1, S_u2, S_h])."""
    fs = _as_fields(prob, fields)
    outs = [np.empty(prob.shape) for _ in range(3)]
    p = prob._c()
    rc = _load().orc_source_mesh(C.byref(p), _fields_ptrs(fs), _fields_ptrs(outs))
    return rc, outs


def run_source(prob: Problem, t0: float, dt: float, nsteps: int, fields):
    """nsteps steps of the source-term scheme (orc_run_source); returns
    (status, fields, accumulated stats)."""
    fs = [f.copy() for f in _as_fields(prob, fields)]
    st = _Stats()
    p = prob._c()
    rc = _load().orc_run_source(C.byref(p), float(t0), float(dt), int(nsteps),
                                _fields_ptrs(fs), C.byref(st))
    return rc, fs, st.as_dict()


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return _load().orc_threads()
