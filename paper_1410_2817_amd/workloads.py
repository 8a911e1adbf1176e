"""Seeded synthetic inputs for the forward semi-Lagrangian step.

This module only *describes* problems: grids, initial fields, velocity-family
parameters, time steps and request streams.  It holds none of the method's
arithmetic (no trajectories, no interpolation), so both the GPU library and the
CPU oracle can be fed from it.  Every random draw comes from
``numpy.random.Generator(PCG64(seed))``.

Shapes follow the pure-advection tests of Sec. 3.1: a cosine hill (eq. "alpha"),
a Gaussian, and a slotted (Zalesak) disc, plus their 3-D analogues.  Arrays are
C-ordered with x fastest; ``shape`` lists the slowest axis first.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Sequence

import numpy as np

# Velocity kinds, numbered as in the C interface.
VEL_UNIFORM, VEL_SOLID_BODY, VEL_SWIRL2D, VEL_DEFORM3D, VEL_FOURIER, VEL_GRIDDED, VEL_CARRIED = range(7)
# Source kinds, numbered as in the C interface.
SRC_NONE, SRC_SHALLOW_WATER = 0, 1


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def coords(shape: Sequence[int], length: Sequence[float] | None = None):
    """Node-centred coordinates x_i = i*h per array axis, broadcastable."""
    d = len(shape)
    length = list(length) if length is not None else [1.0] * d
    out = []
    for a, (n, L) in enumerate(zip(shape, length)):
        x = np.arange(n, dtype=np.float64) * (L / n)
        sh = [1] * d
        sh[a] = n
        out.append(x.reshape(sh))
    return out  # array order: [z,] y, x


def _xyz(shape, length=None):
    """Coordinates as (x, y[, z]) in physical-axis order."""
    c = coords(shape, length)
    return c[::-1]


def gaussian(shape, center, sigma, length=None):
    X = _xyz(shape, length)
    r2 = sum((X[a] - center[a]) ** 2 for a in range(len(shape)))
    return np.broadcast_to(np.exp(-r2 / (2.0 * sigma * sigma)), tuple(shape)).copy()


def cosine_bell(shape, center, radius, length=None):
    """0.5 (1 + cos(pi r / R)) inside r <= R, zero outside (eq. "alpha" has
    R = 0.1 and centre (0.25, 0.5))."""
    X = _xyz(shape, length)
    r = np.sqrt(sum((X[a] - center[a]) ** 2 for a in range(len(shape))))
    v = np.where(r <= radius, 0.5 * (1.0 + np.cos(np.pi * r / radius)), 0.0)
    return np.broadcast_to(v, tuple(shape)).copy()


def slotted_disk(shape, center, radius, slot_width, slot_length, length=None):
    """Zalesak's notched disc (or sphere in 3-D): 1 inside, 0 outside, with a
    slot of the given width along x, cut upward (+y) from the bottom of the
    disc to a depth of slot_length."""
    X = _xyz(shape, length)
    r = np.sqrt(sum((X[a] - center[a]) ** 2 for a in range(len(shape))))
    inside = r <= radius
    slot = (np.abs(X[0] - center[0]) <= 0.5 * slot_width) & (
        X[1] <= center[1] - radius + slot_length)
    v = np.where(inside & ~slot, 1.0, 0.0)
    return np.broadcast_to(v, tuple(shape)).copy()


def disk(shape, center, radius, length=None):
    X = _xyz(shape, length)
    r = np.sqrt(sum((X[a] - center[a]) ** 2 for a in range(len(shape))))
    return np.broadcast_to(np.where(r <= radius, 1.0, 0.0), tuple(shape)).copy()


def fourier_modes(seed: int, dim: int, nmodes: int = 16, kmax: float = 4.0,
                  gen: np.random.Generator | None = None) -> np.ndarray:
    """Random divergence-free flow modes: rows (k[3], a[3], phase).

    k is an integer wave vector with 1 <= |k| <= kmax, a ~ N(0, I) (one
    component in 2-D, three in 3-D) and the phase ~ U[0, 2 pi).  The velocity
    built from them is described with the C velocity descriptor."""
    g = gen if gen is not None else rng(seed)
    kk = int(math.floor(kmax))
    cand = []
    rng_k = range(-kk, kk + 1)
    if dim == 2:
        for ky in rng_k:
            for kx in rng_k:
                n2 = kx * kx + ky * ky
                if 1 <= n2 <= kmax * kmax:
                    cand.append((kx, ky, 0))
    else:
        for kz in rng_k:
            for ky in rng_k:
                for kx in rng_k:
                    n2 = kx * kx + ky * ky + kz * kz
                    if 1 <= n2 <= kmax * kmax:
                        cand.append((kx, ky, kz))
    cand = np.array(cand, dtype=np.float64)
    pick = g.integers(0, len(cand), size=nmodes)
    modes = np.zeros((nmodes, 7))
    modes[:, 0:3] = cand[pick]
    if dim == 2:
        modes[:, 3] = g.standard_normal(nmodes)
    else:
        modes[:, 3:6] = g.standard_normal((nmodes, 3))
    modes[:, 6] = g.uniform(0.0, 2.0 * np.pi, nmodes)
    return modes


def fourier_speed_max(modes: np.ndarray, dim: int, samples: int = 64) -> float:
    """Max-norm speed of the unscaled Fourier flow on a samples^dim lattice of
    the unit box at t = 0.  Used only to choose dt for a target CFL number
    (part of the workload definition, not of the method)."""
    x = np.arange(samples) / samples
    grids = np.meshgrid(*([x] * dim), indexing="ij")  # grids[a] is axis a (x-first)
    u = [np.zeros_like(grids[0]) for _ in range(dim)]
    for md in modes:
        k = md[0:dim]
        k2 = float(np.dot(k, k))
        th = md[6] + 2.0 * np.pi * sum(k[a] * grids[a] for a in range(dim))
        c = np.cos(th) * 2.0 * np.pi / k2
        if dim == 2:
            u[0] += md[3] * c * k[1]
            u[1] -= md[3] * c * k[0]
        else:
            a = md[3:6]
            u[0] += c * (k[1] * a[2] - k[2] * a[1])
            u[1] += c * (k[2] * a[0] - k[0] * a[2])
            u[2] += c * (k[0] * a[1] - k[1] * a[0])
    return float(max(np.abs(ui).max() for ui in u))


@dataclass
class Velocity:
    kind: int
    params: list = field(default_factory=lambda: [0.0] * 8)
    modes: np.ndarray | None = None

    def padded_params(self):
        return list(self.params) + [0.0] * (8 - len(self.params))


@dataclass
class Workload:
    """One advection run: grid, initial fields, velocity, time stepping."""
    name: str
    shape: tuple
    length: tuple
    fields: list          # FP64 numpy arrays, each of `shape`
    velocity: Velocity
    dt: float
    nsteps: int
    t0: float = 0.0
    order_max: int = 2
    limiter: bool = False
    theta: float = 0.25
    value_prec: str = "f64"  # "f64" or "f32" (FP32 values, FP64 positions)
    integrator: int = 0      # 0 RK4, 1 Williamson low-storage RK3
    reconstruct_every: int = 1
    # VEL_GRIDDED: velocity samples on the mesh, components x-first, each an
    # array of `shape` (physical units).
    ugrid: list | None = None
    # Source term: SRC_SHALLOW_WATER with sp = (fc, beta, y0, nu); the fields
    # are then u1, u2, h and the velocity is VEL_CARRIED.
    source: int = SRC_NONE
    sp: tuple = (0.0, 0.0, 0.0, 0.0)

    @property
    def dim(self):
        return len(self.shape)

    @property
    def nfields(self):
        return len(self.fields)

    @property
    def nodes(self):
        return int(np.prod(self.shape))


def sample_velocity(wl: "Workload", t: float = 0.0) -> list:
    """The analytic velocity of workload wl at the mesh nodes at time t
    (components x-first, each an array of wl.shape): the input of a gridded
    velocity run.  Part of the problem definition, not of the method."""
    d = wl.dim
    X = _xyz(wl.shape, wl.length)  # x, y[, z], broadcastable
    L = list(wl.length)[::-1]      # physical-axis order
    p = wl.velocity.padded_params()
    kind = wl.velocity.kind
    zero = np.zeros(wl.shape)
    full = lambda a: np.broadcast_to(np.asarray(a, dtype=np.float64), wl.shape).copy()
    pi = np.pi
    if kind == VEL_UNIFORM:
        u = [full(p[a]) for a in range(d)]
    elif kind == VEL_SOLID_BODY:
        u = [full(-p[0] * (X[1] - p[2])), full(p[0] * (X[0] - p[1]))] + ([zero.copy()] if d == 3 else [])
    elif kind == VEL_SWIRL2D:
        c = np.cos(pi * t / p[0])
        u = [full(p[1] * np.sin(pi * X[0]) ** 2 * np.sin(2 * pi * X[1]) * c),
             full(-p[1] * np.sin(pi * X[1]) ** 2 * np.sin(2 * pi * X[0]) * c)]
    elif kind == VEL_DEFORM3D:
        c = np.cos(pi * t / p[0])
        s1 = [np.sin(pi * X[a]) for a in range(3)]
        s2 = [np.sin(2 * pi * X[a]) for a in range(3)]
        u = [full(2 * p[1] * s1[0] ** 2 * s2[1] * s2[2] * c),
             full(-p[1] * s2[0] * s1[1] ** 2 * s2[2] * c),
             full(-p[1] * s2[0] * s2[1] * s1[2] ** 2 * c)]
    elif kind == VEL_FOURIER:
        u = [zero.copy() for _ in range(d)]
        for md in wl.velocity.modes:
            k = md[0:d]
            k2 = float(np.dot(k, k))
            th = md[6] + 2 * pi * sum(k[a] * X[a] / L[a] for a in range(d))
            g = [np.cos(th) * 2 * pi * k[a] / L[a] / k2 for a in range(d)]
            if d == 2:
                u[0] = u[0] + md[3] * g[1]
                u[1] = u[1] - md[3] * g[0]
            else:
                a_ = md[3:6]
                u[0] = u[0] + g[1] * a_[2] - g[2] * a_[1]
                u[1] = u[1] + g[2] * a_[0] - g[0] * a_[2]
                u[2] = u[2] + g[0] * a_[1] - g[1] * a_[0]
        u = [full(ui * p[0]) for ui in u]
    else:
        raise ValueError("no analytic velocity for kind %d" % kind)
    return u


def gridded(wl: "Workload", order: int = 2, t: float = 0.0) -> "Workload":
    """Workload wl with its velocity replaced by the mesh samples of its
    analytic velocity at time t (held fixed), interpolated with the Z-spline
    of the given order."""
    import dataclasses
    return dataclasses.replace(wl, name=wl.name + "_gridded%d" % order,
                               velocity=Velocity(VEL_GRIDDED, [float(order)]),
                               ugrid=sample_velocity(wl, t))


def burgers(n: int = 256, dim: int = 2, t_end: float = 0.3, cfl: float = 0.5,
            value_prec: str = "f64") -> Workload:
    """Burgers' equation Du/Dt = 0 with the radial initial velocity of the
    paper's shock test (Sec. 3): u = exp(-150 (r - 0.2)^2) (x - c) / r for
    r = |x - c| > 0.001 (c the box centre), 0 otherwise; the velocity is
    carried by the fields (fields 0..dim-1), limiter on, Z2.  Max speed 1, so
    the step is at most cfl h; the run ends at t_end exactly."""
    shape = (n,) * dim
    X = _xyz(shape)
    rel = [X[a] - 0.5 for a in range(dim)]
    r = np.sqrt(sum(q * q for q in rel))
    amp = np.where(r > 0.001, np.exp(-150.0 * (r - 0.2) ** 2) / np.maximum(r, 1e-300), 0.0)
    fs = [np.broadcast_to(amp * rel[a], shape).astype(np.float64).copy() for a in range(dim)]
    nsteps = int(math.ceil(t_end * n / cfl - 1e-9))
    return Workload("burgers%dd_%d_%s" % (dim, n, value_prec), shape, (1.0,) * dim, fs,
                    Velocity(VEL_CARRIED), dt=t_end / nsteps, nsteps=nsteps,
                    order_max=2, limiter=True, value_prec=value_prec)


def kelvin_fields(shape, t: float, amp: float, f0: float, x0: float = 0.5,
                  y0: float = 0.5) -> list:
    """The equatorial Kelvin wave of the linearised shallow-water system
    (eq. "kelvin"): h = u1 = exp(-f0 y^2/2) K(x - t), u2 = 0, with
    K(s) = amp exp(-f0 s^2/2), y measured from the equator y0 and s from x0,
    periodic in x (nearest image) on the unit box.  Returns [u1, u2, h]."""
    X = _xyz(shape)
    s = X[0] - x0 - t
    s = s - np.round(s)
    y = X[1] - y0
    h = np.broadcast_to(amp * np.exp(-0.5 * f0 * s * s) * np.exp(-0.5 * f0 * y * y),
                        tuple(shape)).astype(np.float64).copy()
    return [h.copy(), np.zeros(tuple(shape)), h]


def kelvin(n: int = 256, amp: float = 1e-4, f0: float = 250.0, nu: float = 0.0,
           t_end: float = 1.0, cfl: float = 0.5, value_prec: str = "f64",
           limiter: bool = False) -> Workload:
    """Shallow-water Kelvin-wave test of Sec. 3 (eq. "nlsw" with the equatorial
    beta plane f = f0 (y - 0.5) on the unit box, bi-periodic): the initial
    state is the Kelvin wave at t = 0 with K(x) = amp exp(-f0 x^2/2) centred on
    x = 0.5.  amp = 1e-4, nu = 0 is the linear convergence test (the exact
    solution travels east at unit speed, so at t = 1 it is back where it
    started); amp = 0.5, nu = 5e-4 is the non-linear run.  Fields u1, u2, h;
    carried velocity; Z2.  dt = t_end / nsteps with the step at most cfl h (unit
    gravity-wave speed) and, with viscosity, at most h^2 / (16 nu): the
    five-point viscous operator reaches 16 nu (1 + h) / h^2 on the grid's
    finest mode, and the RK3 stability interval on the negative axis ends near
    2.5, so the bound holds while 1 + h <= 2."""
    shape = (n, n)
    fs = kelvin_fields(shape, 0.0, amp, f0)
    h = 1.0 / n
    step = cfl * h
    if nu > 0.0:
        step = min(step, h * h / (16.0 * nu))
    nsteps = int(math.ceil(t_end / step - 1e-9))
    tag = "kelvin" if amp <= 1e-2 else "kelvin_nonlinear"
    return Workload("%s_%d_%s" % (tag, n, value_prec), shape, (1.0, 1.0), fs,
                    Velocity(VEL_CARRIED), dt=t_end / nsteps, nsteps=nsteps,
                    order_max=2, limiter=limiter, value_prec=value_prec,
                    integrator=1, source=SRC_SHALLOW_WATER, sp=(0.0, f0, 0.5, nu))


def solid_body_gaussian(n: int = 64, steps: int = 100, order_max: int = 2) -> Workload:
    """2-D solid-body rotation of a Gaussian hump (centre (0.5, 0.75), sigma
    0.05) about (0.5, 0.5) at angular speed 2 pi: `steps` steps make one turn.
    RK4 trajectories, FP64, limiter off."""
    shape = (n, n)
    f = gaussian(shape, (0.5, 0.75), 0.05)
    vel = Velocity(VEL_SOLID_BODY, [2.0 * np.pi, 0.5, 0.5])
    return Workload("sbr_gaussian_%d" % n, shape, (1.0, 1.0), [f], vel,
                    dt=1.0 / steps, nsteps=steps, order_max=order_max,
                    limiter=False, value_prec="f64")


def solid_body_cosine_hill(n: int = 50, steps: int = 200, order_max: int = 2,
                           limiter: bool = False) -> Workload:
    """The cosine hill of eq. "alpha" (radius 0.1 at (0.25, 0.5)) under
    solid-body rotation about the domain centre, one turn in `steps` steps."""
    shape = (n, n)
    f = cosine_bell(shape, (0.25, 0.5), 0.1)
    vel = Velocity(VEL_SOLID_BODY, [2.0 * np.pi, 0.5, 0.5])
    return Workload("sbr_cosine_hill_%d" % n, shape, (1.0, 1.0), [f], vel,
                    dt=1.0 / steps, nsteps=steps, order_max=order_max,
                    limiter=limiter, value_prec="f64")


def swirl_three_fields(n: int = 1024, cfl: float = 4.0, period: float = 5.0,
                       value_prec: str = "f32", nsteps: int | None = None) -> Workload:
    """2-D reversing swirl (period T = 5, max speed 1) carrying a slotted disc
    (R 0.15 at (0.5, 0.75), slot 0.05 x 0.25), a cosine bell (R 0.15 at
    (0.25, 0.5)) and a Gaussian (sigma 0.05 at (0.5, 0.25)).  dt = cfl * h;
    a full period is T / dt steps.  Limiter on."""
    shape = (n, n)
    fs = [slotted_disk(shape, (0.5, 0.75), 0.15, 0.05, 0.25),
          cosine_bell(shape, (0.25, 0.5), 0.15),
          gaussian(shape, (0.5, 0.25), 0.05)]
    vel = Velocity(VEL_SWIRL2D, [period, 1.0])
    dt = cfl / n
    full = int(round(period / dt))
    return Workload("swirl2d_%d_%s" % (n, value_prec), shape, (1.0, 1.0), fs, vel,
                    dt=dt, nsteps=full if nsteps is None else nsteps,
                    order_max=2, limiter=True, value_prec=value_prec)


def fourier3d_three_fields(n: int = 256, seed: int = 0, cfl: float = 2.0,
                           nsteps: int = 50, value_prec: str = "f32") -> Workload:
    """3-D periodic box, divergence-free flow from 16 random Fourier modes
    (|k| <= 4, amplitudes N(0,1)/|k|^2), carrying a slotted sphere, a cosine
    bell and a Gaussian.  dt gives max-speed CFL = cfl at t = 0."""
    shape = (n, n, n)
    fs = [slotted_disk(shape, (0.5, 0.75, 0.5), 0.15, 0.05, 0.25),
          cosine_bell(shape, (0.25, 0.5, 0.5), 0.15),
          gaussian(shape, (0.5, 0.25, 0.5), 0.05)]
    modes = fourier_modes(seed, 3)
    umax = fourier_speed_max(modes, 3)
    vel = Velocity(VEL_FOURIER, [1.0], modes)
    return Workload("fourier3d_%d_%s" % (n, value_prec), shape, (1.0, 1.0, 1.0), fs,
                    vel, dt=cfl / (n * umax), nsteps=nsteps, order_max=2,
                    limiter=True, value_prec=value_prec)


def deform3d_slotted_sphere(n: int = 512, period: float = 3.0, nsteps: int = 60,
                            value_prec: str = "f64") -> Workload:
    """3-D deformational flow (period T = 3, max speed 2) carrying one slotted
    sphere (R 0.15 at (0.35, 0.35, 0.35)); dt = 3h/2 (CFL 3)."""
    shape = (n, n, n)
    fs = [slotted_disk(shape, (0.35, 0.35, 0.35), 0.15, 0.05, 0.25)]
    vel = Velocity(VEL_DEFORM3D, [period, 1.0])
    return Workload("deform3d_%d_%s" % (n, value_prec), shape, (1.0, 1.0, 1.0), fs,
                    vel, dt=1.5 / n, nsteps=nsteps, order_max=2, limiter=True,
                    value_prec=value_prec)


def uniform_translation(shape, velocity, dt, fields, nsteps=1, order_max=2,
                        limiter=False, value_prec="f64", length=None) -> Workload:
    """Uniform flow: the building block of the identity, shift and
    polynomial-reproduction checks."""
    length = tuple(length) if length is not None else (1.0,) * len(shape)
    vel = Velocity(VEL_UNIFORM, list(velocity))
    return Workload("uniform", tuple(shape), length, list(fields), vel, dt=dt,
                    nsteps=nsteps, order_max=order_max, limiter=limiter,
                    value_prec=value_prec)


# ---------------------------------------------------------------------------
# Serving stream: many independent 2-D problems arriving over time.

SERVING_SIDES = (128, 256, 512, 1024, 2048)


@dataclass
class Component:
    kind: str            # "gaussian" or "disk"
    center: tuple
    size: float          # sigma or radius


@dataclass
class Request:
    """One serving request.  Field values are built on demand from the drawn
    components (numpy for the oracle, torch on the device for the server)."""
    rid: int
    arrival: float        # seconds after the stream starts
    n: int
    nsteps: int
    dt: float
    modes: np.ndarray
    fields_spec: list     # per field: list of Component

    @property
    def shape(self):
        return (self.n, self.n)

    @property
    def nfields(self):
        return len(self.fields_spec)

    @property
    def nodes(self):
        return self.n * self.n

    def fields(self):
        out = []
        for comps in self.fields_spec:
            f = np.zeros(self.shape)
            for c in comps:
                if c.kind == "gaussian":
                    f += gaussian(self.shape, c.center, c.size)
                else:
                    f += disk(self.shape, c.center, c.size)
            out.append(f)
        return out

    def fields_torch(self, device, dtype):
        """The same fields evaluated with torch on `device`."""
        import torch
        x = torch.arange(self.n, device=device, dtype=torch.float64) / self.n
        X = x[None, :]
        Y = x[:, None]
        out = []
        for comps in self.fields_spec:
            f = torch.zeros(self.shape, device=device, dtype=torch.float64)
            for c in comps:
                r2 = (X - c.center[0]) ** 2 + (Y - c.center[1]) ** 2
                if c.kind == "gaussian":
                    f += torch.exp(-r2 / (2.0 * c.size * c.size))
                else:
                    f += (r2.sqrt() <= c.size).to(torch.float64)
            out.append(f.to(dtype).contiguous())
        return out

    @property
    def workload(self) -> Workload:
        vel = Velocity(VEL_FOURIER, [1.0], self.modes)
        return Workload("req%d_%d" % (self.rid, self.n), self.shape, (1.0, 1.0),
                        self.fields(), vel, dt=self.dt, nsteps=self.nsteps, order_max=2,
                        limiter=True, value_prec="f32")


def _components(g: np.random.Generator) -> list:
    """1-3 components, each a Gaussian (sigma ~ U[0.02, 0.1]) or a step disc
    (R ~ U[0.05, 0.2]) at a uniform random centre."""
    comps = []
    for _ in range(int(g.integers(1, 4))):
        c = tuple(g.uniform(0.2, 0.8, 2))
        if g.uniform() < 0.5:
            comps.append(Component("gaussian", c, float(g.uniform(0.02, 0.1))))
        else:
            comps.append(Component("disk", c, float(g.uniform(0.05, 0.2))))
    return comps


def serving_request(g: np.random.Generator, rid: int, arrival: float,
                    sides=SERVING_SIDES, cfl: float = 2.0,
                    steps_range=(10, 50)) -> Request:
    n = int(g.choice(np.asarray(sides)))
    nf = int(g.integers(1, 5))
    nsteps = int(g.integers(steps_range[0], steps_range[1] + 1))
    spec = [_components(g) for _ in range(nf)]
    modes = fourier_modes(0, 2, gen=g)
    umax = fourier_speed_max(modes, 2)
    return Request(rid, arrival, n, nsteps, cfl / (n * umax), modes, spec)


def serving_stream(seed: int = 0, count: int = 512, rate: float = 100.0,
                   sides=SERVING_SIDES, steps_range=(10, 50)) -> list:
    """`count` requests with Poisson arrivals at `rate` per second."""
    g = rng(seed)
    gaps = g.exponential(1.0 / rate, count)
    t = np.cumsum(gaps) - gaps[0]
    return [serving_request(g, i, float(t[i]), sides=sides, steps_range=steps_range)
            for i in range(count)]
