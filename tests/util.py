"""Helpers shared by the GPU parity tests: build oracle problems and GPU grids
from the same seeded workload, compare results."""
import numpy as np


def oracle_problem(orc, wl, **kw):
    return orc.Problem(wl.shape, wl.nfields, wl.length, order_max=wl.order_max,
                       limiter=wl.limiter, theta=wl.theta, integrator=wl.integrator,
                       vel_kind=wl.velocity.kind, vp=wl.velocity.padded_params(),
                       modes=wl.velocity.modes, ugrid=getattr(wl, "ugrid", None),
                       src_kind=getattr(wl, "source", 0),
                       sp=list(getattr(wl, "sp", (0.0,) * 4)), **kw)


def stored_values(wl):
    """Inputs as the GPU stores them (rounded to FP32 for the split form), in
    FP64 so the oracle sees exactly the same numbers."""
    if wl.value_prec == "f32":
        return [np.asarray(f, dtype=np.float32).astype(np.float64) for f in wl.fields]
    return [np.asarray(f, dtype=np.float64) for f in wl.fields]


def l1_rel(got, want):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    return float(np.abs(got - want).sum() / max(np.abs(want).sum(), 1e-300))


def linf(got, want):
    return float(np.abs(np.asarray(got, np.float64) - np.asarray(want, np.float64)).max())


def tol(wl):
    """Parity tolerance on relative L1: 1e-12 for FP64 runs, 1e-5 for FP32
    values with FP64 positions."""
    return 1e-5 if wl.value_prec == "f32" else 1e-12
