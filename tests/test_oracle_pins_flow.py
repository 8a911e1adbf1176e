"""More pins of the CPU oracle: the jump criterion where the two one-sided
slopes differ, the structure of the reversing swirl and the 3-D deformational
flow, and the sampled full-size step against the ordinary step.

Each check is built from a mathematical property, not from a second copy of
the oracle's formula, so that a slip in the oracle fails one of them.
"""
import math

import numpy as np
import pytest

from paper_1410_2817_amd import workloads as W


# --------------------------------------------------------------------------
# Jump criterion of Sec. 2.3 on geometric profiles.
#
# On h_i = r^i the differences are D2 = r^(i-1) (r-1)^2, D+ = r^i (r-1),
# D- = r^(i-1) (r-1).  The criterion |D2| > theta max(|D+|, |D-|) fires iff
#   r > 1:  (r-1)/r > theta,  i.e. r > 1/(1-theta)    (4/3 for theta 1/4),
#   r < 1:  (1-r)   > theta,  i.e. r < 1 - theta      (3/4 for theta 1/4),
# whereas the smaller slope in place of the larger would fire from r > 1+theta
# and r < 1/(1+theta).  The ratios below sit between the two thresholds.

def _geometric(shape, axis, r):
    """r^i along array axis `axis` (i the index there), constant across it."""
    n = shape[axis]
    prof = r ** np.arange(n, dtype=np.float64)
    view = [1] * len(shape)
    view[axis] = n
    return np.broadcast_to(prof.reshape(view), shape).copy()


@pytest.mark.parametrize("shape", [(6, 40), (5, 6, 40)])
@pytest.mark.parametrize("theta", [0.25, 0.1])
def test_jump_criterion_on_geometric_profiles(orc, shape, theta):
    up = 1.0 / (1.0 - theta)   # growth threshold of the criterion
    down = 1.0 - theta         # decay threshold
    cases = [  # (ratio, fires)
        (0.5 * (1.0 + theta) + 0.5 * up, False),   # between 1+theta and 1/(1-theta)
        (up + 0.05, True),
        (0.5 / (1.0 + theta) + 0.5 * down, False),  # between 1/(1+theta) and 1-theta
        (down - 0.05, True),
        (1.0 + 0.5 * theta, False),                 # gentle growth: never
    ]
    dim = len(shape)
    for axis in range(dim):
        # Sizes along the tested axis are long enough to keep the periodic wrap
        # (where the profile jumps back) away from the checked interior nodes.
        sh = list(shape)
        sh[axis], sh[-1] = sh[-1], sh[axis]
        sh = tuple(sh)
        prob = orc.Problem(sh, 1, theta=theta)
        n = sh[axis]
        for r, fires in cases:
            f = _geometric(sh, axis, r)
            fl = orc.flags(prob, [f])
            inner = np.take(fl, np.arange(2, n - 2), axis=axis)
            assert np.all(inner == (1 if fires else 0)), (axis, r, fires, theta)


def test_jump_criterion_takes_the_larger_slope(orc):
    # h = (0, 1, 2.3) around the middle node: D2 = 0.3, D+ = 1.3, D- = 1.
    # 0.3 > 0.25 * 1.3 is false, so the node is not flagged; with the smaller
    # slope (0.3 > 0.25) it would be.  Mirrored: the same.
    prob = orc.Problem((3, 8), 1)
    for row in ([0.0, 1.0, 2.3], [2.3, 1.0, 0.0]):
        f = np.zeros((3, 8))
        f[:, 2:5] = row
        f[:, 5:] = row[-1]
        assert orc.flag(prob, f, (3, 1)) == 0
    # curvature just above a quarter of the larger slope fires
    f = np.zeros((3, 8))
    f[:, 2:5] = [0.0, 1.0, 2.34]
    f[:, 5:] = 2.34
    assert orc.flag(prob, f, (3, 1)) == 1


def test_jump_criterion_is_affine_invariant_and_axis_or(orc):
    # Adding a constant or scaling the field leaves every flag unchanged; a
    # node fires when any axis fires.
    g = np.random.Generator(np.random.PCG64(11))
    shape = (12, 14)
    f = g.standard_normal(shape)
    prob = orc.Problem(shape, 1)
    base = orc.flags(prob, [f])
    assert np.array_equal(base, orc.flags(prob, [3.5 * f - 7.0]))
    assert np.array_equal(base, orc.flags(prob, [-0.25 * f]))
    fx = _geometric(shape, 1, 1.45)  # fires along x in the interior
    fy = np.ones(shape)
    both = orc.flags(prob, [fx * fy])
    assert both[:, 2:-2].all()
    assert not orc.flags(prob, [np.ones(shape) * 2.0]).any()


# --------------------------------------------------------------------------
# Reversing swirl and 3-D deformational flow (LeVeque-type test flows).

def _div(orc, prob, x, t, eps=1e-4):
    """Divergence by fourth-order central differences."""
    d = len(x)
    s = 0.0
    for a in range(d):
        e = np.zeros(d)
        e[a] = eps
        u = lambda y: orc.velocity(prob, y, t)[a]
        s += (-u(x + 2 * e) + 8 * u(x + e) - 8 * u(x - e) + u(x - 2 * e)) / (12 * eps)
    return s


def _grad_scale(orc, prob, x, t, eps=1e-4):
    d = len(x)
    m = 0.0
    for a in range(d):
        e = np.zeros(d)
        e[a] = eps
        m = max(m, np.abs(orc.velocity(prob, x + e, t) - orc.velocity(prob, x - e, t)).max()
                / (2 * eps))
    return m


@pytest.mark.parametrize("kind", ["swirl", "deform3d"])
def test_test_flows_are_divergence_free(orc, kind):
    if kind == "swirl":
        prob = orc.Problem((16, 16), 1, vel_kind=orc.VEL_SWIRL2D, vp=[5.0, 1.0])
        dim = 2
    else:
        prob = orc.Problem((8, 8, 8), 1, vel_kind=orc.VEL_DEFORM3D, vp=[3.0, 1.0])
        dim = 3
    g = np.random.Generator(np.random.PCG64(5))
    big = 0.0
    for _ in range(20):
        x = g.uniform(0.0, 1.0, dim)
        t = float(g.uniform(0.0, 1.0))
        scale = _grad_scale(orc, prob, x, t)
        big = max(big, scale)
        assert abs(_div(orc, prob, x, t)) <= 1e-9 * max(scale, 1.0), (x, t)
    assert big > 1.0  # the flow is not trivially zero


def test_swirl_is_the_curl_of_its_stream_function(orc):
    # psi = (p1 / pi) sin^2(pi x) sin^2(pi y) cos(pi t / T); u = psi_y, v = -psi_x.
    T, p1 = 5.0, 1.3
    prob = orc.Problem((16, 16), 1, vel_kind=orc.VEL_SWIRL2D, vp=[T, p1])

    def psi(x, t):
        return p1 / math.pi * math.sin(math.pi * x[0]) ** 2 * math.sin(math.pi * x[1]) ** 2 \
            * math.cos(math.pi * t / T)

    eps = 1e-5
    g = np.random.Generator(np.random.PCG64(6))
    for _ in range(10):
        x = g.uniform(0, 1, 2)
        t = float(g.uniform(0, T))
        u = orc.velocity(prob, x, t)
        py = (psi(x + [0, eps], t) - psi(x - [0, eps], t)) / (2 * eps)
        px = (psi(x + [eps, 0], t) - psi(x - [eps, 0], t)) / (2 * eps)
        assert abs(u[0] - py) < 1e-8 and abs(u[1] + px) < 1e-8


@pytest.mark.parametrize("kind", ["swirl", "deform3d"])
def test_test_flows_reverse_in_time_and_respect_the_box(orc, kind):
    if kind == "swirl":
        T, dim = 5.0, 2
        prob = orc.Problem((16, 16), 1, vel_kind=orc.VEL_SWIRL2D, vp=[T, 1.0])
    else:
        T, dim = 3.0, 3
        prob = orc.Problem((8, 8, 8), 1, vel_kind=orc.VEL_DEFORM3D, vp=[T, 1.0])
    g = np.random.Generator(np.random.PCG64(7))
    for _ in range(10):
        x = g.uniform(0, 1, dim)
        t = float(g.uniform(0, T))
        u = orc.velocity(prob, x, t)
        # the time factor is odd about T/2: the flow runs backwards
        assert np.allclose(orc.velocity(prob, x, T - t), -u, rtol=0, atol=1e-14)
        # periodic in every axis with period 1
        for a in range(dim):
            e = np.zeros(dim)
            e[a] = 1.0
            assert np.allclose(orc.velocity(prob, x + e, t), u, rtol=0, atol=1e-13)
            # no flow across the faces x_a = 0 of the unit box
            y = x.copy()
            y[a] = 0.0
            assert abs(orc.velocity(prob, y, t)[a]) < 1e-15
    # at t = T/2 the flow stops
    x = np.full(dim, 0.3)
    assert np.abs(orc.velocity(prob, x, 0.5 * T)).max() < 1e-15


@pytest.mark.parametrize("kind", ["swirl", "deform3d"])
def test_trajectories_return_after_one_period(orc, kind):
    # Every material point is carried back to its start at t = T; the RK4
    # return error shrinks at fourth order while the half-period excursion is
    # of order one.
    if kind == "swirl":
        T, n = 5.0, 16
        prob = orc.Problem((n, n), 1, vel_kind=orc.VEL_SWIRL2D, vp=[T, 1.0])
        nodes = [(4, 9), (11, 3), (8, 8)]
    else:
        T, n = 3.0, 8
        prob = orc.Problem((n, n, n), 1, vel_kind=orc.VEL_DEFORM3D, vp=[T, 1.0])
        nodes = [(2, 3, 5), (6, 1, 4)]
    errs = []
    for steps in (100, 200):
        dt = T / steps
        worst, far = 0.0, 0.0
        for node in nodes:
            d = np.zeros(len(node))
            for s in range(steps):
                d = orc.trajectory(prob, node, s * dt, dt, d)
                if s == steps // 2 - 1:
                    far = max(far, np.abs(d).max())
            worst = max(worst, np.abs(d).max())
        assert far > 0.5  # cells: the points travel far at mid-period
        errs.append(worst)
    assert errs[1] < 5e-6 and errs[0] / errs[1] > 12.0, errs


# --------------------------------------------------------------------------
# The sampled step (trajectories the search touches integrated on demand,
# flags evaluated on demand) is the reference of the full-size GPU checks; it
# must be the ordinary step exactly, node for node.

def _problem(orc, wl, **kw):
    return orc.Problem(wl.shape, wl.nfields, wl.length, order_max=wl.order_max,
                       limiter=wl.limiter, theta=wl.theta, integrator=wl.integrator,
                       vel_kind=wl.velocity.kind, vp=wl.velocity.padded_params(),
                       modes=wl.velocity.modes, **kw)


def _sampled_cases():
    sw = W.swirl_three_fields(48, value_prec="f64")
    sw_rk3 = W.swirl_three_fields(40, value_prec="f64")
    sw_rk3.integrator = 1
    sw_z1 = W.swirl_three_fields(40, value_prec="f64")
    sw_z1.order_max = 1
    de = W.deform3d_slotted_sphere(20)
    fo = W.fourier3d_three_fields(16)
    bu = W.burgers(40)
    return [
        ("swirl_t07", sw, 0.7, 1, None),
        ("swirl_k2", sw, 1.9, 2, None),
        ("swirl_rk3", sw_rk3, 0.3, 1, None),
        ("swirl_z1_k2", sw_z1, 2.6, 2, None),
        ("swirl_shard", sw, 0.45, 1, (7, 100)),
        ("deform3d", de, 0.4, 1, None),
        ("deform3d_k2", de, 1.1, 2, None),
        ("fourier3d", fo, 0.0, 1, None),
        ("fourier3d_shard", fo, 0.2, 1, (3, -5, 9)),
        ("burgers", bu, 0.0, 1, None),
    ]


@pytest.mark.parametrize("case", _sampled_cases(), ids=lambda c: c[0])
def test_sampled_step_equals_the_step(orc, case):
    _, wl, t, ksteps, offset = case
    prob = _problem(orc, wl, offset=offset)
    fields = [np.asarray(f, np.float64) for f in wl.fields]
    if wl.velocity.kind == orc.VEL_CARRIED:
        prob.ugrid = fields[:wl.dim]
    # the ordinary path: trajectories over ksteps sub-steps, then reconstruct
    rc, want, st = orc.run(prob, t, wl.dt, ksteps, fields, kevery=ksteps)
    assert rc == 0 and st["search_fail"] == 0 and st["newton_fail"] == 0
    nodes = np.arange(wl.nodes, dtype=np.int64)
    rc2, got, st2 = orc.step_sampled(prob, t, wl.dt, fields, nodes, ksteps=ksteps)
    assert rc2 == 0
    for f in range(wl.nfields):
        assert np.array_equal(got[:, f], want[f].ravel()), f
    assert st2["order_hist"] == st["order_hist"]
    # a strided subset returns the same values at its nodes
    sub = nodes[::7]
    rc3, part, _ = orc.step_sampled(prob, t, wl.dt, fields, sub, ksteps=ksteps)
    assert rc3 == 0 and np.array_equal(part, got[::7])
    # the run moved things: not an identity
    assert any(not np.array_equal(want[f], fields[f]) for f in range(wl.nfields))


# --------------------------------------------------------------------------
# FP32 storage between steps (the values the FP32-value form carries).

def test_f32_storage_run_is_steps_with_rounding_between(orc):
    wl = W.swirl_three_fields(40, value_prec="f32")
    prob = _problem(orc, wl)
    f0 = [np.asarray(f, np.float32).astype(np.float64) for f in wl.fields]
    rc, got, _ = orc.run(prob, 0.3, wl.dt, 5, f0, store="f32")
    assert rc == 0
    cur = [f.copy() for f in f0]
    for s in range(5):
        rc, cur, _ = orc.run(prob, 0.3 + s * wl.dt, wl.dt, 1, cur)
        assert rc == 0
        cur = [np.asarray(f, np.float32).astype(np.float64) for f in cur]
    for a, b in zip(got, cur):
        assert np.array_equal(a, b)
        assert np.array_equal(a, a.astype(np.float32).astype(np.float64))
    # without rounding the values are not all FP32 numbers
    rc, plain, _ = orc.run(prob, 0.3, wl.dt, 5, f0)
    assert any(not np.array_equal(p, p.astype(np.float32).astype(np.float64)) for p in plain)
    assert max(np.abs(p - q).max() for p, q in zip(plain, got)) < 1e-5
