"""Pins of the oracle's source-term path (the right-hand side S_i of eq.
"momento", finite differences on the reference mesh, Williamson's RK3 along
the lattice) against closed forms and the paper's Kelvin-wave test.

Closed forms used: the symbols of the centred finite-difference rules on a
Fourier mode, the stability polynomial 1 + z + z^2/2 + z^3/6 that every
three-stage third-order Runge-Kutta scheme has on a linear autonomous system,
the derivatives of the Z-splines at their knots (eq. "matchder"), and the exact
Kelvin wave (eq. "kelvin").  None of them re-derives the oracle's own code.
"""
import math

import numpy as np
import pytest

from paper_1410_2817_amd import workloads as W


def _sw(orc, shape, m=2, fc=0.0, beta=0.0, y0=0.5, nu=0.0, nfields=3, limiter=False):
    return orc.Problem(shape, nfields, (1.0, 1.0), order_max=m, limiter=limiter,
                       integrator=orc.RK3_WILLIAMSON, vel_kind=orc.VEL_CARRIED,
                       src_kind=orc.SRC_SHALLOW_WATER, sp=[fc, beta, y0, nu])


def _rk3_power(L, dt, n):
    """P(dt L)^n for the RK3 stability polynomial P(z) = 1 + z + z^2/2 + z^3/6."""
    Z = dt * np.asarray(L, dtype=np.float64)
    I = np.eye(Z.shape[0])
    P = I + Z + Z @ Z / 2.0 + Z @ Z @ Z / 6.0
    return np.linalg.matrix_power(P, n)


def _d1_symbol(M, theta, h):
    # i * this = the centred first-derivative rule applied to exp(i k x)
    if M == 1:
        return math.sin(theta) / h
    return (8.0 * math.sin(theta) - math.sin(2.0 * theta)) / (6.0 * h)


def _d2_symbol(M, theta, h):
    # the centred second-derivative rule applied to exp(i k x), divided by it
    if M == 1:
        return (2.0 * math.cos(theta) - 2.0) / (h * h)
    return (-15.0 + 16.0 * math.cos(theta) - math.cos(2.0 * theta)) / (6.0 * h * h)


def _one_sided_derivs(f, x, side, order):
    hs = side * 1e-3 * np.arange(0, 8)
    ys = np.array([f(x + h) for h in hs])
    c = np.polyfit(hs, ys, 7)[::-1]
    return [c[p] * math.factorial(p) for p in range(order + 1)]


# --------------------------------------------------------------------------
# Finite-difference rules

@pytest.mark.parametrize("m,p", [(1, 1), (2, 1), (2, 2)])
def test_fd_weights_are_the_zspline_knot_derivatives(orc, m, p):
    """Eq. "matchder": the p-th derivative of the order-m Z-spline interpolant
    at a knot is the (2m+1)-point centred finite difference, so the rule's
    weight of sample j is Z_m^(p)(-j)."""
    c = orc.fd_weights(m, p)
    f = lambda x: orc.zspline(m, x)
    for j in range(-m, m + 1):
        d = _one_sided_derivs(f, float(-j), +1, m)[p]
        assert abs(c[j + m] - d) < 2e-6, (m, p, j, c[j + m], d)


@pytest.mark.parametrize("M", [1, 2])
def test_fd_weights_exact_on_polynomials(orc, M):
    # A (2M+1)-point rule is exact up to degree 2M, not beyond (degree 2M+1
    # for the symmetric second derivative).
    for p in (1, 2):
        c = orc.fd_weights(M, p)
        ks = np.arange(-M, M + 1, dtype=np.float64)
        for q in range(0, 2 * M + 1):
            want = math.factorial(q) if q == p else 0.0
            assert abs(float(np.sum(c * ks ** q)) - want) < 1e-13
        top = 2 * M + 2 if p == 2 else 2 * M + 1
        assert abs(float(np.sum(c * ks ** top))) > 1e-3


@pytest.mark.parametrize("M", [1, 2])
def test_source_on_the_mesh_converges_to_the_analytic_rhs(orc, M):
    """The mesh right-hand side of eq. "nlsw" (with viscosity and a beta plane)
    tends to the analytic one at the order of the rules: 2 (three points) or 4
    (five points).  Mixed derivatives, the (1 + h) factors and the grad h
    products all enter."""
    fc, beta, nu = 3.0, 40.0, 0.02
    errs = []
    for n in (32, 64):
        shape = (n, n)
        x, y = W._xyz(shape)
        k = 2.0 * np.pi
        X, Y = k * x, k * y
        u = 0.3 * np.sin(X) * np.cos(Y) + 0.0 * y
        v = 0.2 * np.cos(X) * np.sin(2 * Y)
        h = 0.1 * np.sin(X + Y)
        ux, uy = 0.3 * k * np.cos(X) * np.cos(Y), -0.3 * k * np.sin(X) * np.sin(Y)
        uxx = uyy = -0.3 * k * k * np.sin(X) * np.cos(Y)
        uxy = -0.3 * k * k * np.cos(X) * np.sin(Y)
        vx, vy = -0.2 * k * np.sin(X) * np.sin(2 * Y), 0.4 * k * np.cos(X) * np.cos(2 * Y)
        vxx = -0.2 * k * k * np.cos(X) * np.sin(2 * Y)
        vyy = -0.8 * k * k * np.cos(X) * np.sin(2 * Y)
        vxy = -0.4 * k * k * np.sin(X) * np.cos(2 * Y)
        hx = hy = 0.1 * k * np.cos(X + Y)
        f = fc + beta * (y - 0.5)
        # grad u + grad u^T, its divergence weighted by (1 + h)
        s_h = -(1 + h) * (ux + vy)
        s_u = -hx + f * v + nu * ((1 + h) * (2 * uxx + uyy + vxy) + hx * 2 * ux + hy * (uy + vx))
        s_v = -hy - f * u + nu * ((1 + h) * (vxx + 2 * vyy + uxy) + hx * (vx + uy) + hy * 2 * vy)
        fields = [np.broadcast_to(a, shape).copy() for a in (u, v, h)]
        rc, S = orc.source_mesh(_sw(orc, shape, m=M, fc=fc, beta=beta, nu=nu), fields)
        assert rc == 0
        want = [np.broadcast_to(a, shape) for a in (s_u, s_v, s_h)]
        errs.append(max(float(np.abs(S[c] - want[c]).max()) for c in range(3)))
    order = math.log2(errs[0] / errs[1])
    assert order > (3.7 if M == 2 else 1.8), (errs, order)


# --------------------------------------------------------------------------
# Whole steps against closed forms

@pytest.mark.parametrize("m", [1, 2])
def test_linear_standing_wave_follows_the_discrete_dispersion_relation(orc, m):
    """Linear gravity waves (f = 0, nu = 0, tiny amplitude), the paper's
    dispersion test: h = A cos(kx), u = 0 evolves as the 2x2 system
    a' = -k* b, b' = k* a (h = a cos, u1 = b sin) with k* the symbol of the
    first-derivative rule, advanced by the RK3 polynomial."""
    ny, nx, kk, A = 8, 32, 2, 1e-9
    shape = (ny, nx)
    hx = 1.0 / nx
    x, _ = W._xyz(shape)
    kap = 2.0 * np.pi * kk
    hfield = np.broadcast_to(A * np.cos(kap * x), shape).copy()
    z = np.zeros(shape)
    dt, n = 0.5 * hx, 20
    rc, out, st = orc.run_source(_sw(orc, shape, m=m), 0.0, dt, n, [z, z.copy(), hfield])
    assert rc == 0 and st["search_fail"] == 0
    ks = _d1_symbol(m, kap * hx, hx)
    a, b = _rk3_power([[0.0, -ks], [ks, 0.0]], dt, n) @ np.array([A, 0.0])
    xb = np.broadcast_to(x, shape)
    assert np.abs(out[2] - a * np.cos(kap * xb)).max() < 1e-6 * A
    assert np.abs(out[0] - b * np.sin(kap * xb)).max() < 1e-6 * A
    assert np.abs(out[1]).max() < 1e-6 * A
    # and the discrete frequency is below the exact one (k* < k), as a
    # centred rule must give
    assert ks < kap


def test_inertial_oscillation_is_the_rk3_rotation(orc):
    """Uniform fields on an f-plane: u' = f u2, u2' = -f u1 (the -f u_perp term
    with u_perp = (-u2, u1)), h unchanged; the lattice translates by a
    non-integer shift and a uniform field reconstructs to itself."""
    shape = (12, 16)
    fc, dt, n = 7.0, 0.01, 25
    u0 = [np.full(shape, 0.3), np.zeros(shape), np.full(shape, 0.05)]
    rc, out, _ = orc.run_source(_sw(orc, shape, fc=fc), 0.0, dt, n, u0)
    assert rc == 0
    want = _rk3_power([[0.0, fc], [-fc, 0.0]], dt, n) @ np.array([0.3, 0.0])
    assert np.abs(out[0] - want[0]).max() < 1e-13
    assert np.abs(out[1] - want[1]).max() < 1e-13
    assert np.abs(out[2] - 0.05).max() < 1e-13


@pytest.mark.parametrize("m", [1, 2])
def test_viscous_shear_decays_with_the_second_derivative_symbol(orc, m):
    """u1 = U sin(2 pi k y), u2 = h = 0, nu > 0: the viscous term is nu u1_yy
    and nothing else moves; the lattice rows slide along x, which leaves an
    x-uniform field unchanged."""
    ny, nx, kk, U, nu = 32, 16, 3, 0.2, 0.01
    shape = (ny, nx)
    _, y = W._xyz(shape)
    hy = 1.0 / ny
    u1 = np.broadcast_to(U * np.sin(2 * np.pi * kk * y), shape).copy()
    z = np.zeros(shape)
    dt, n = 0.01, 10
    rc, out, st = orc.run_source(_sw(orc, shape, m=m, nu=nu), 0.0, dt, n, [u1, z, z.copy()])
    assert rc == 0 and st["search_fail"] == 0
    lam = _d2_symbol(m, 2 * np.pi * kk * hy, hy)
    g = _rk3_power([[nu * lam]], dt, n)[0, 0]
    assert np.abs(out[0] - g * u1).max() < 1e-12
    assert np.abs(out[1]).max() < 1e-13 and np.abs(out[2]).max() < 1e-13
    assert g < 1.0


def test_compressional_wave_is_damped_by_twice_nu(orc):
    """A compressional mode feels nu (u_xx + d_x div u) = 2 nu u_xx: with
    h = a cos(kx), u1 = b sin(kx) the linear system is a' = -k* b,
    b' = k* a + 2 nu l* b (k*, l* the rule symbols)."""
    ny, nx, kk, A, nu = 8, 32, 3, 1e-9, 0.02
    shape = (ny, nx)
    hx = 1.0 / nx
    x, _ = W._xyz(shape)
    kap = 2.0 * np.pi * kk
    hfield = np.broadcast_to(A * np.cos(kap * x), shape).copy()
    z = np.zeros(shape)
    dt, n = 0.5 * hx, 16
    rc, out, _ = orc.run_source(_sw(orc, shape, nu=nu), 0.0, dt, n, [z, z.copy(), hfield])
    assert rc == 0
    ks, ls = _d1_symbol(2, kap * hx, hx), _d2_symbol(2, kap * hx, hx)
    a, b = _rk3_power([[0.0, -ks], [ks, 2.0 * nu * ls]], dt, n) @ np.array([A, 0.0])
    xb = np.broadcast_to(x, shape)
    assert np.abs(out[2] - a * np.cos(kap * xb)).max() < 1e-6 * A
    assert np.abs(out[0] - b * np.sin(kap * xb)).max() < 1e-6 * A


def test_passive_field_is_carried_like_burgers(orc):
    """With uniform velocity and no Coriolis force the velocity has no source,
    so a fourth (passive) field moves exactly as under the plain carried
    velocity: the same straight paths, the same reconstruction."""
    shape = (24, 20)
    g = W.gaussian(shape, (0.4, 0.6), 0.1)
    fs = [np.full(shape, 0.3), np.full(shape, -0.2), np.zeros(shape), g]
    dt, n = 0.013, 4
    rc, out, _ = orc.run_source(_sw(orc, shape, nfields=4), 0.0, dt, n, fs)
    assert rc == 0
    plain = orc.Problem(shape, 4, (1.0, 1.0), order_max=2, vel_kind=orc.VEL_CARRIED)
    rc2, ref, _ = orc.run(plain, 0.0, dt, n, fs)
    assert rc2 == 0
    assert np.abs(out[3] - ref[3]).max() < 1e-13
    assert np.abs(out[0] - 0.3).max() < 1e-14 and np.abs(out[1] + 0.2).max() < 1e-14


def test_time_integration_is_third_order_along_moving_lattices(orc):
    """A strong pressure gradient (h a Gaussian of height 0.2) in a uniform
    stream (0.3, 0.1): the lattice moves several cells but hardly deforms, so
    the reconstruction error does not depend on dt and Richardson differences
    of runs at dt, dt/2, dt/4 show the order of the time integration.  It is
    near three only if each stage uses the lattice nodes' own stage velocity and
    the right-hand side interpolated at their stage positions (either slip
    drops it to one)."""
    n = 48
    shape = (n, n)
    g = W.gaussian(shape, (0.5, 0.5), 0.1) * 0.2
    fs = [np.full(shape, 0.3), np.full(shape, 0.1), g]
    prob = _sw(orc, shape)
    res = []
    for ns in (8, 16, 32):
        rc, out, st = orc.run_source(prob, 0.0, 0.08 / ns, ns, fs)
        assert rc == 0 and st["search_fail"] == 0
        res.append(out)
    orders = []
    for c in range(3):
        d = [float(np.abs(res[i][c] - res[i + 1][c]).max()) for i in range(2)]
        orders.append(math.log2(d[0] / d[1]))
    assert min(orders[:2]) > 2.6 and orders[2] > 2.0, orders


@pytest.mark.slow
def test_kelvin_wave_converges_at_third_order(orc):
    """Sec. 3, shallow water: the equatorial Kelvin wave (eq. "kelvin") with
    f0 = 250 and amplitude 1e-4; the relative L2 error of h against the exact
    wave falls at least at third order under refinement with dt = h/2."""
    errs = []
    for n in (32, 64, 128):
        wl = W.kelvin(n, amp=1e-4, t_end=0.25)
        prob = _sw(orc, wl.shape, fc=wl.sp[0], beta=wl.sp[1], y0=wl.sp[2], nu=wl.sp[3])
        rc, out, st = orc.run_source(prob, 0.0, wl.dt, wl.nsteps, wl.fields)
        assert rc == 0 and st["search_fail"] == 0
        ex = W.kelvin_fields(wl.shape, 0.25, 1e-4, 250.0)
        errs.append(math.sqrt(float(((out[2] - ex[2]) ** 2).sum() / (ex[2] ** 2).sum())))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) > 3.0, (errs, orders)
    assert errs[-1] < 5e-4
