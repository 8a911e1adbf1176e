/*
 * Plain FP64 CPU oracle of the forward semi-Lagrangian (FSL) step of
 * Becerra-Sagredo, Malaga & Mandujano, "Moments Preserving and high-resolution
 * Semi-Lagrangian Advection Scheme".
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct reference
 * that the GPU library is checked against.  Only the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load it.  It shares no source,
 * header, table or helper with the GPU library.
 *
 * What one step computes (Sec. 2 of the paper):
 *   1. every lattice node starts on its reference-mesh node and is carried along
 *      its trajectory dx/dt = u(x,t)                       (eqs. "momento", "vel")
 *   2. each lattice node is flagged when the jump criterion fires (Sec. 2.3)
 *   3. for every reference-mesh node: find the deformed material element that
 *      holds it, invert the multilinear (Z0) element map with Newton's method
 *      (Sec. 2.2, eq. "mapping1"), pick the interpolation order so that no
 *      flagged point enters the stencil (Sec. 2.3) and evaluate the tensor
 *      product Z-spline sum of eq. "multiZ" with the cardinal basis of the
 *      Appendix.
 * With a source term (orc_run_source) the lattice nodes also carry their
 * values, integrated with Williamson's low-storage RK3 against a right-hand
 * side taken by finite differences on the mesh from the stage fields.
 *
 * Conventions (readings of points the paper leaves open):
 *   - node-centred periodic grid, x_i = i*h, h = L/N, values stored x fastest;
 *   - lattice displacements are kept in cell units, positions are never wrapped;
 *   - the multi-dimensional jump criterion applies the 1-D test along each axis
 *     and flags the node if any axis fires; it is written in multiplied-out form
 *     |D2| > theta*max(|D+|,|D-|) so that flat data is never flagged;
 *   - flags are per field;
 *   - the element search starts at floor(i - d_i), where d_i is the displacement
 *     of the lattice node with the same index (the point "opposite to the
 *     velocity"), and moves one cell per axis toward the side indicated by an
 *     out-of-range local coordinate.
 *
 * Everything is FP64.  The cardinal basis alone is evaluated in long double and
 * rounded once, because the Appendix polynomials on 2<=|x|<=3 cancel terms of
 * size ~350 and plain FP64 evaluation would leave ~1e-13 absolute error, too
 * close to the tolerances this oracle is meant to certify.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_DIM 3
#define ORC_MAX_FIELDS 8

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ESEARCH = -4, ORC_ENEWTON = -5 };
enum { ORC_RK4 = 0, ORC_RK3_WILLIAMSON = 1 };
enum { ORC_SRC_NONE = 0, ORC_SRC_SHALLOW_WATER = 1 };
enum {
  ORC_VEL_UNIFORM = 0,
  ORC_VEL_SOLID_BODY = 1,
  ORC_VEL_SWIRL2D = 2,
  ORC_VEL_DEFORM3D = 3,
  ORC_VEL_FOURIER = 4,
  ORC_VEL_GRIDDED = 5,
  ORC_VEL_CARRIED = 6
};

/* Problem description, mirrored field by field by the ctypes binding. */
typedef struct {
  int dim;
  int nfields;
  int64_t n[3];
  double len[3];
  int order_max;      /* 0, 1 or 2: Z0, Z1, Z2 */
  int limiter;        /* 0 off, 1 on */
  double theta;       /* jump threshold, 0.25 in the paper */
  int integrator;     /* ORC_RK4 or ORC_RK3_WILLIAMSON */
  int vel_kind;
  double vp[8];       /* velocity parameters, see orc_velocity */
  int nmodes;
  const double *modes;  /* nmodes x 7: k[3], a[3], phase */
  int newton_max_iter;
  double newton_tol;    /* on max |delta xi| */
  int walk_max;
  double eps_inside;    /* slack on the unit cube when accepting an element */
  int scan_radius;      /* half-width of the fallback scan box */
  const double *ugrid[3]; /* GRIDDED: velocity components on the mesh nodes;
                           * CARRIED: set internally to the fields at reset */
  int src_kind;         /* ORC_SRC_*: right-hand side S_i of eq. "momento" */
  double sp[4];         /* SHALLOW_WATER: fc, beta, y0, nu (see orc_source_mesh) */
  int64_t offset[3];    /* index of node 0 in a larger lattice (a shard): the
                         * trajectory of node i starts at (i + offset) h */
} orc_problem;

typedef struct {
  int64_t nodes;
  int64_t search_fail;
  int64_t newton_fail;
  int64_t order_hist[3];  /* per field-node */
  int64_t flagged;        /* flagged lattice points, summed over fields */
  int64_t walk_steps;     /* extra cells visited beyond the first */
  int64_t newton_iters;
} orc_stats;

/* ------------------------------------------------------------------------- */
/* Cardinal Z-spline basis (Appendix).  Z0 is the linear hat, the degree-1,
 * C0 member of the family (the paper names it but does not print it).        */
double orc_zspline(int m, double xd) {
  long double a = fabsl((long double)xd);
  long double a2 = a * a, a3 = a2 * a, a4 = a3 * a, a5 = a4 * a;
  /* Each piece is written over a common integer denominator so that the
   * knots (integer a) evaluate exactly. */
  switch (m) {
    case 0:
      return a <= 1.0L ? (double)(1.0L - a) : 0.0;
    case 1:
      if (a <= 1.0L) return (double)((2.0L - 5.0L * a2 + 3.0L * a3) / 2.0L);
      if (a <= 2.0L) return (double)((2.0L - a) * (2.0L - a) * (1.0L - a) / 2.0L);
      return 0.0;
    case 2:
      /* 1 - 15/12 a^2 - 35/12 a^3 + 63/12 a^4 - 25/12 a^5 */
      if (a <= 1.0L)
        return (double)((12.0L - 15.0L * a2 - 35.0L * a3 + 63.0L * a4 -
                         25.0L * a5) / 12.0L);
      /* -4 + 75/4 a - 245/8 a^2 + 545/24 a^3 - 63/8 a^4 + 25/24 a^5 */
      if (a <= 2.0L)
        return (double)((-96.0L + 450.0L * a - 735.0L * a2 + 545.0L * a3 -
                         189.0L * a4 + 25.0L * a5) / 24.0L);
      /* 18 - 153/4 a + 255/8 a^2 - 313/24 a^3 + 21/8 a^4 - 5/24 a^5 */
      if (a <= 3.0L)
        return (double)((432.0L - 918.0L * a + 765.0L * a2 - 313.0L * a3 +
                         63.0L * a4 - 5.0L * a5) / 24.0L);
      return 0.0;
    default:
      return NAN;
  }
}

/* Weights of the 2m+2 nodes r-m..r+m+1 for a point r+t (eq. "multiZ" along one
 * axis): w[k+m] = Z_m(t - k).                                                */
void orc_weights(int m, double t, double *w) {
  for (int k = -m; k <= m + 1; ++k) w[k + m] = orc_zspline(m, t - (double)k);
}

/* Periodic index in [0, n). */
static int64_t orc_wrap(int64_t i, int64_t n) {
  int64_t r = i % n;
  return r < 0 ? r + n : r;
}

/* Tensor-product cardinal Z-spline interpolation of order m (eq. "multiZ") of
 * ng mesh fields g[0..ng-1] at the physical point x, periodic; out[c] receives
 * the value of field c.                                                      */
static void orc_zinterp(const orc_problem *P, int m, int ng,
                        const double *const *g, const double *x, double *out) {
  int64_t r[3] = {0, 0, 0};
  double w[3][6];
  for (int a = 0; a < 3; ++a)
    for (int k = 0; k < 6; ++k) w[a][k] = a < P->dim ? 0.0 : 1.0;
  for (int a = 0; a < P->dim; ++a) {
    const double s = x[a] / (P->len[a] / (double)P->n[a]);
    r[a] = (int64_t)floor(s);
    orc_weights(m, s - (double)r[a], w[a]);
  }
  for (int c = 0; c < ng; ++c) out[c] = 0.0;
  const int np = 2 * m + 2;
  const int nz = P->dim == 3 ? np : 1;
  for (int kz = 0; kz < nz; ++kz)
    for (int ky = 0; ky < np; ++ky)
      for (int kx = 0; kx < np; ++kx) {
        const int64_t ix = orc_wrap(r[0] - m + kx, P->n[0]);
        const int64_t iy = orc_wrap(r[1] - m + ky, P->n[1]);
        const int64_t iz = P->dim == 3 ? orc_wrap(r[2] - m + kz, P->n[2]) : 0;
        const int64_t lin = ix + P->n[0] * (iy + P->n[1] * iz);
        const double wt = w[0][kx] * w[1][ky] * (P->dim == 3 ? w[2][kz] : 1.0);
        for (int c = 0; c < ng; ++c) out[c] += wt * g[c][lin];
      }
}

/* ------------------------------------------------------------------------- */
/* Prescribed velocity fields u(x,t) in physical coordinates.
 *   UNIFORM     u = (p0, p1, p2)
 *   SOLID_BODY  u = p0 * (-(y - p2), x - p1, 0)            rotation about (p1,p2)
 *   SWIRL2D     u =  p1 sin^2(pi x) sin(2 pi y) cos(pi t / p0)
 *               v = -p1 sin^2(pi y) sin(2 pi x) cos(pi t / p0)
 *   DEFORM3D    u =  2 p1 sin^2(pi x) sin(2 pi y) sin(2 pi z) c
 *               v =   -p1 sin(2 pi x) sin^2(pi y) sin(2 pi z) c
 *               w =   -p1 sin(2 pi x) sin(2 pi y) sin^2(pi z) c,  c = cos(pi t/p0)
 *   FOURIER     divergence-free sum of modes (k, a, phase), theta = 2 pi k.x/L + phase
 *               2-D: psi = sum a0/|k|^2 sin(theta), u = (d psi/dy, -d psi/dx)
 *               3-D: A = sum a/|k|^2 sin(theta),     u = curl A
 *               all scaled by p0.
 *   GRIDDED     samples of u on the mesh nodes (ugrid), interpolated with
 *               the Z-spline of order p0
 *   CARRIED     u is transported with the fields (fields 0..dim-1 are its
 *               components) and has no right-hand side (Burgers' equation
 *               Du/Dt = 0): each lattice node keeps the velocity it had at
 *               the last reset, so it moves on a straight line; see
 *               orc_trajectory.                                              */
void orc_velocity(const orc_problem *P, const double *x, double t, double *u) {
  const double pi = M_PI;
  u[0] = u[1] = u[2] = 0.0;
  switch (P->vel_kind) {
    case ORC_VEL_UNIFORM:
      for (int a = 0; a < P->dim; ++a) u[a] = P->vp[a];
      break;
    case ORC_VEL_SOLID_BODY:
      u[0] = -P->vp[0] * (x[1] - P->vp[2]);
      u[1] = P->vp[0] * (x[0] - P->vp[1]);
      break;
    case ORC_VEL_SWIRL2D: {
      double c = cos(pi * t / P->vp[0]);
      double sx = sin(pi * x[0]), sy = sin(pi * x[1]);
      u[0] = P->vp[1] * sx * sx * sin(2.0 * pi * x[1]) * c;
      u[1] = -P->vp[1] * sy * sy * sin(2.0 * pi * x[0]) * c;
      break;
    }
    case ORC_VEL_DEFORM3D: {
      double c = cos(pi * t / P->vp[0]);
      double sx = sin(pi * x[0]), sy = sin(pi * x[1]), sz = sin(pi * x[2]);
      double s2x = sin(2.0 * pi * x[0]), s2y = sin(2.0 * pi * x[1]),
             s2z = sin(2.0 * pi * x[2]);
      u[0] = 2.0 * P->vp[1] * sx * sx * s2y * s2z * c;
      u[1] = -P->vp[1] * s2x * sy * sy * s2z * c;
      u[2] = -P->vp[1] * s2x * s2y * sz * sz * c;
      break;
    }
    case ORC_VEL_FOURIER: {
      for (int q = 0; q < P->nmodes; ++q) {
        const double *md = P->modes + 7 * q;
        double th = md[6], k2 = 0.0;
        for (int a = 0; a < P->dim; ++a) {
          th += 2.0 * pi * md[a] * x[a] / P->len[a];
          k2 += md[a] * md[a];
        }
        /* d/dx_a sin(theta) = cos(theta) * 2 pi k_a / L_a */
        double g[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < P->dim; ++a)
          g[a] = cos(th) * 2.0 * pi * md[a] / P->len[a] / k2;
        if (P->dim == 2) {
          u[0] += md[3] * g[1];
          u[1] -= md[3] * g[0];
        } else {
          /* curl(a f) = grad f x a */
          u[0] += g[1] * md[5] - g[2] * md[4];
          u[1] += g[2] * md[3] - g[0] * md[5];
          u[2] += g[0] * md[4] - g[1] * md[3];
        }
      }
      for (int a = 0; a < P->dim; ++a) u[a] *= P->vp[0];
      break;
    }
    case ORC_VEL_GRIDDED:
      /* Velocity given on the reference mesh, interpolated at x with the
       * tensor-product cardinal Z-spline of order vp[0] (eq. "multiZ" applied
       * to the velocity samples; periodic). */
      orc_zinterp(P, (int)P->vp[0], P->dim, P->ugrid, x, u);
      break;
    default:
      u[0] = u[1] = u[2] = NAN;
  }
}

/* ------------------------------------------------------------------------- */
/* Trajectory of one lattice node over [t, t+dt] (Sec. 2: integration along the
 * path of a material element).  disp is the displacement in cell units since
 * the last reset and is updated in place.                                   */
void orc_trajectory(const orc_problem *P, const int64_t *node, double t,
                    double dt, double *disp) {
  int d = P->dim;
  double h[3] = {1.0, 1.0, 1.0}, x[3] = {0.0, 0.0, 0.0}, y[3] = {0.0, 0.0, 0.0};
  double k1[3], k2[3], k3[3], k4[3];
  for (int a = 0; a < d; ++a) {
    h[a] = P->len[a] / (double)P->n[a];
    x[a] = ((double)(node[a] + P->offset[a]) + disp[a]) * h[a];
  }
  if (P->vel_kind == ORC_VEL_CARRIED) {
    /* Du/Dt = 0: the node's own velocity (its field values at the reset,
     * held in ugrid) is constant along its path; every integrator is exact. */
    int64_t lin = 0;
    for (int a = d - 1; a >= 0; --a) lin = lin * P->n[a] + node[a];
    for (int a = 0; a < d; ++a) disp[a] += dt * P->ugrid[a][lin] / h[a];
    return;
  }
  if (P->integrator == ORC_RK4) {
    orc_velocity(P, x, t, k1);
    for (int a = 0; a < d; ++a) y[a] = x[a] + 0.5 * dt * k1[a];
    orc_velocity(P, y, t + 0.5 * dt, k2);
    for (int a = 0; a < d; ++a) y[a] = x[a] + 0.5 * dt * k2[a];
    orc_velocity(P, y, t + 0.5 * dt, k3);
    for (int a = 0; a < d; ++a) y[a] = x[a] + dt * k3[a];
    orc_velocity(P, y, t + dt, k4);
    for (int a = 0; a < d; ++a)
      disp[a] += dt * (k1[a] + 2.0 * k2[a] + 2.0 * k3[a] + k4[a]) / 6.0 / h[a];
  } else {
    /* Low-storage third-order Runge-Kutta of Williamson (1980), the 2N-storage
     * scheme with A = (0, -5/9, -153/128), B = (1/3, 15/16, 8/15) and stage
     * times c = (0, 1/3, 3/4):  q = A_s q + dt u(x, t + c_s dt);  x += B_s q. */
    static const double A[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
    static const double B[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};
    static const double C[3] = {0.0, 1.0 / 3.0, 3.0 / 4.0};
    double q[3] = {0.0, 0.0, 0.0}, dx[3] = {0.0, 0.0, 0.0}, u[3];
    for (int s = 0; s < 3; ++s) {
      for (int a = 0; a < d; ++a) y[a] = x[a] + dx[a];
      orc_velocity(P, y, t + C[s] * dt, u);
      for (int a = 0; a < d; ++a) {
        q[a] = A[s] * q[a] + dt * u[a];
        dx[a] += B[s] * q[a];
      }
    }
    for (int a = 0; a < d; ++a) disp[a] += dx[a] / h[a];
  }
}

static int64_t total_nodes(const orc_problem *P) {
  int64_t c = 1;
  for (int a = 0; a < P->dim; ++a) c *= P->n[a];
  return c;
}

static void unflatten(const orc_problem *P, int64_t lin, int64_t *idx) {
  for (int a = 0; a < P->dim; ++a) {
    idx[a] = lin % P->n[a];
    lin /= P->n[a];
  }
}

static int64_t wrap(int64_t i, int64_t n) {
  int64_t r = i % n;
  return r < 0 ? r + n : r;
}

static int64_t flatten_wrapped(const orc_problem *P, const int64_t *idx) {
  int64_t lin = 0;
  for (int a = P->dim - 1; a >= 0; --a) lin = lin * P->n[a] + wrap(idx[a], P->n[a]);
  return lin;
}

/* All lattice nodes; disp is SoA, disp[a * Ntot + node]. */
void orc_trajectories(const orc_problem *P, double t, double dt, double *disp) {
  int64_t N = total_nodes(P);
#pragma omp parallel for schedule(static)
  for (int64_t lin = 0; lin < N; ++lin) {
    int64_t idx[3];
    double dd[3] = {0.0, 0.0, 0.0};
    unflatten(P, lin, idx);
    for (int a = 0; a < P->dim; ++a) dd[a] = disp[a * N + lin];
    orc_trajectory(P, idx, t, dt, dd);
    for (int a = 0; a < P->dim; ++a) disp[a * N + lin] = dd[a];
  }
}

/* ------------------------------------------------------------------------- */
/* Jump criterion of Sec. 2.3 at one lattice point for one field.             */
int orc_flag(const orc_problem *P, const double *field, const int64_t *node) {
  int64_t nb[3];
  double hc = field[flatten_wrapped(P, node)];
  for (int a = 0; a < P->dim; ++a) {
    memcpy(nb, node, sizeof(nb));
    nb[a] = node[a] + 1;
    double hp = field[flatten_wrapped(P, nb)];
    nb[a] = node[a] - 1;
    double hm = field[flatten_wrapped(P, nb)];
    double d2 = hp - 2.0 * hc + hm;
    double dp = hp - hc;
    double dm = hc - hm;
    if (fabs(d2) > P->theta * fmax(fabs(dp), fabs(dm))) return 1;
  }
  return 0;
}

/* Flags of every lattice point, bit f for field f.                           */
void orc_flags(const orc_problem *P, const double *const *fields, uint8_t *flags) {
  int64_t N = total_nodes(P);
#pragma omp parallel for schedule(static)
  for (int64_t lin = 0; lin < N; ++lin) {
    int64_t idx[3];
    unflatten(P, lin, idx);
    uint8_t b = 0;
    for (int f = 0; f < P->nfields; ++f)
      if (orc_flag(P, fields[f], idx)) b |= (uint8_t)(1u << f);
    flags[lin] = b;
  }
}

/* ------------------------------------------------------------------------- */
/* Element localisation (Sec. 2.2).
 *
 * The element with lower vertex r has vertices r+e, e in {0,1}^d, at lattice
 * positions (r+e) + disp(r+e).  Its Z0 map is the multilinear interpolant
 *     x(xi) = sum_e X_e prod_a phi_{e_a}(xi_a),  phi_0 = 1 - s, phi_1 = s,
 * whose Taylor series about a vertex is finite (eq. "mapping1").  With
 * V_e = X_e - x' (the target mesh point) the equation x(xi) = x' becomes
 * F(xi) = sum_e V_e prod_a phi = 0, solved by Newton's method from the
 * solution of its linear part.  Displacements are supplied by a callback so
 * that the sampled mode can integrate trajectories on demand.               */
typedef void (*orc_disp_fn)(void *ctx, const int64_t *node, double *d);

static int solve_dxd(int d, double J[3][3], const double *b, double *x) {
  /* Cramer's rule. */
  if (d == 1) {
    if (J[0][0] == 0.0) return -1;
    x[0] = b[0] / J[0][0];
    return 0;
  }
  if (d == 2) {
    double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    if (det == 0.0 || !isfinite(det)) return -1;
    x[0] = (b[0] * J[1][1] - J[0][1] * b[1]) / det;
    x[1] = (J[0][0] * b[1] - b[0] * J[1][0]) / det;
    return 0;
  }
  double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
               J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
               J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
  if (det == 0.0 || !isfinite(det)) return -1;
  for (int c = 0; c < 3; ++c) {
    double M[3][3];
    memcpy(M, J, sizeof(M));
    for (int r = 0; r < 3; ++r) M[r][c] = b[r];
    double dc = M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) -
                M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
                M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
    x[c] = dc / det;
  }
  return 0;
}

/* F(xi) and its Jacobian J[i][a] = dF_i/dxi_a for vertex offsets V[e][i]. */
static void element_map(int d, double V[8][3], const double *xi, double *F,
                        double J[3][3]) {
  for (int i = 0; i < 3; ++i) {
    F[i] = 0.0;
    for (int a = 0; a < 3; ++a) J[i][a] = 0.0;
  }
  for (int e = 0; e < (1 << d); ++e) {
    double phi[3], dphi[3];
    for (int a = 0; a < d; ++a) {
      int bit = (e >> a) & 1;
      phi[a] = bit ? xi[a] : 1.0 - xi[a];
      dphi[a] = bit ? 1.0 : -1.0;
    }
    double w = 1.0;
    for (int a = 0; a < d; ++a) w *= phi[a];
    for (int i = 0; i < d; ++i) F[i] += V[e][i] * w;
    for (int a = 0; a < d; ++a) {
      double g = dphi[a];
      for (int b = 0; b < d; ++b)
        if (b != a) g *= phi[b];
      for (int i = 0; i < d; ++i) J[i][a] += V[e][i] * g;
    }
  }
}

/* Newton solve of the Z0 map of the element with lower vertex r for the mesh
 * point `target`.  Returns 1 when Newton converged (xi holds the solution),
 * 0 when only the solution of the linear part is available (xi holds that),
 * -1 when even the linear part is singular.                                 */
static int element_solve(const orc_problem *P, orc_disp_fn get_disp, void *ctx,
                         const int64_t *target, const int64_t *r, double *xi,
                         int *newton_iters) {
  int d = P->dim;
  double V[8][3];
  for (int e = 0; e < (1 << d); ++e) {
    int64_t v[3];
    double dv[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < d; ++a) v[a] = r[a] + ((e >> a) & 1);
    get_disp(ctx, v, dv);
    for (int a = 0; a < d; ++a) V[e][a] = (double)(v[a] - target[a]) + dv[a];
  }
  /* Linear part of the expansion about vertex r: J0 xi = -V_0. */
  double J0[3][3], rhs[3], xl[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < d; ++i) {
    rhs[i] = -V[0][i];
    for (int a = 0; a < d; ++a) J0[i][a] = V[1 << a][i] - V[0][i];
  }
  if (solve_dxd(d, J0, rhs, xl) != 0) return -1;
  double x[3] = {xl[0], xl[1], xl[2]};
  for (int it = 0; it < P->newton_max_iter; ++it) {
    double F[3], J[3][3], dl[3];
    element_map(d, V, x, F, J);
    ++*newton_iters;
    if (solve_dxd(d, J, F, dl) != 0) break;
    double mx = 0.0;
    for (int a = 0; a < d; ++a) {
      x[a] -= dl[a];
      mx = fmax(mx, fabs(dl[a]));
    }
    if (!isfinite(mx)) break;
    if (mx <= P->newton_tol) {
      for (int a = 0; a < d; ++a) xi[a] = x[a];
      return 1;
    }
  }
  for (int a = 0; a < d; ++a) xi[a] = xl[a];
  return 0;
}

static int in_cube(const orc_problem *P, const double *xi) {
  for (int a = 0; a < P->dim; ++a)
    if (!(xi[a] >= -P->eps_inside && xi[a] <= 1.0 + P->eps_inside)) return 0;
  return 1;
}

/* Locate mesh node `target` (integer cell coordinates).  On success r holds
 * the lower vertex (unwrapped) and xi the local coordinates.
 *
 * Search (Sec. 2.2): start in the cell below target - d(target) and, while
 * the local coordinates fall outside the unit cube, move one cell per axis
 * toward the indicated side.  A cell is the host only when Newton converges
 * to a point of its unit cube (the "bounded mapping" of the paper); where
 * Newton does not converge, the root of the linear part of the map points the
 * way.  Where the lattice is so distorted that this walk stalls or cycles
 * (e.g. the corners of a periodic box swept by a non-periodic solid-body
 * rotation, or a strongly twisted element whose linear root lies inside but
 * whose Newton iteration wanders off), the cells of the box of half-width
 * scan_radius around the start cell are tried in order, x fastest, and the
 * first that holds the point is taken.  Failure is reported as ORC_ENEWTON
 * if some visited cell had its linear root inside but no Newton solution,
 * else as ORC_ESEARCH.                                                      */
int orc_locate_cb(const orc_problem *P, orc_disp_fn get_disp, void *ctx,
                  const int64_t *target, int64_t *r, double *xi,
                  int *walk_steps, int *newton_iters) {
  int d = P->dim;
  double d0[3] = {0.0, 0.0, 0.0};
  int64_t start[3] = {0, 0, 0};
  int newton_trouble = 0;
  get_disp(ctx, target, d0);
  for (int a = 0; a < d; ++a) start[a] = r[a] = (int64_t)floor((double)target[a] - d0[a]);
  *walk_steps = 0;
  *newton_iters = 0;
  for (int walk = 0; walk < P->walk_max; ++walk) {
    double x[3] = {0.0, 0.0, 0.0};
    int rc = element_solve(P, get_disp, ctx, target, r, x, newton_iters);
    if (rc < 0) break;
    if (in_cube(P, x)) {
      if (rc == 1) {
        for (int a = 0; a < d; ++a) xi[a] = x[a];
        return ORC_OK;
      }
      newton_trouble = 1;
      break;
    }
    for (int a = 0; a < d; ++a) {
      if (x[a] < -P->eps_inside) r[a] -= 1;
      else if (x[a] > 1.0 + P->eps_inside) r[a] += 1;
    }
    ++*walk_steps;
  }
  int W = P->scan_radius, span = 2 * P->scan_radius + 1;
  int64_t cnt = 1;
  for (int a = 0; a < d; ++a) cnt *= span;
  for (int64_t q = 0; q < cnt; ++q) {
    int64_t qq = q;
    double x[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < d; ++a) {
      r[a] = start[a] - W + qq % span;
      qq /= span;
    }
    int rc = element_solve(P, get_disp, ctx, target, r, x, newton_iters);
    if (in_cube(P, x)) {
      if (rc == 1) {
        for (int a = 0; a < d; ++a) xi[a] = x[a];
        ++*walk_steps;
        return ORC_OK;
      }
      if (rc == 0) newton_trouble = 1;
    }
  }
  return newton_trouble ? ORC_ENEWTON : ORC_ESEARCH;
}

/* Displacement providers: a stored SoA array, or on-demand trajectories. */
typedef struct {
  const orc_problem *P;
  const double *disp;
  int64_t ntot;
} array_ctx;

static void disp_from_array(void *vctx, const int64_t *node, double *d) {
  array_ctx *c = (array_ctx *)vctx;
  int64_t lin = flatten_wrapped(c->P, node);
  for (int a = 0; a < c->P->dim; ++a) d[a] = c->disp[a * c->ntot + lin];
}

typedef struct {
  const orc_problem *P;
  double t, dt;
  int ksteps;
} traj_ctx;

static void disp_on_demand(void *vctx, const int64_t *node, double *d) {
  traj_ctx *c = (traj_ctx *)vctx;
  int64_t w[3] = {0, 0, 0};
  for (int a = 0; a < c->P->dim; ++a) w[a] = wrap(node[a], c->P->n[a]);
  d[0] = d[1] = d[2] = 0.0;
  for (int s = 0; s < c->ksteps; ++s)
    orc_trajectory(c->P, w, c->t + s * c->dt, c->dt, d);
}

int orc_locate(const orc_problem *P, const double *disp, const int64_t *target,
               int64_t *r, double *xi, int *walk_steps, int *newton_iters) {
  array_ctx c = {P, disp, total_nodes(P)};
  return orc_locate_cb(P, disp_from_array, &c, target, r, xi, walk_steps,
                       newton_iters);
}

/* ------------------------------------------------------------------------- */
/* Reconstruction at one mesh node (Sec. 2.1-2.3).  flag_of(f, node) reports
 * the jump flag of a lattice point.  Writes nfields outputs, returns status. */
typedef int (*orc_flag_fn)(void *ctx, int f, const int64_t *node);

static int node_reconstruct(const orc_problem *P, orc_disp_fn get_disp,
                            void *dctx, orc_flag_fn flag_of, void *fctx,
                            const double *const *fin, const int64_t *target,
                            double *out, int8_t *order_out, orc_stats *st) {
  int d = P->dim;
  int64_t r[3] = {0, 0, 0};
  double xi[3] = {0.0, 0.0, 0.0};
  int ws = 0, ni = 0;
  int rc = orc_locate_cb(P, get_disp, dctx, target, r, xi, &ws, &ni);
  if (st) {
    st->walk_steps += ws;
    st->newton_iters += ni;
  }
  if (rc != ORC_OK) {
    for (int f = 0; f < P->nfields; ++f) {
      out[f] = NAN;
      if (order_out) order_out[f] = -1;
    }
    if (st) {
      if (rc == ORC_ESEARCH) st->search_fail++;
      else st->newton_fail++;
    }
    return rc;
  }
  for (int f = 0; f < P->nfields; ++f) {
    /* Order: reduce m while a flagged point lies in the stencil. */
    int m = P->order_max;
    while (P->limiter && m > 0) {
      int hit = 0;
      int64_t span = 2 * m + 2, cnt = 1;
      for (int a = 0; a < d; ++a) cnt *= span;
      for (int64_t q = 0; q < cnt && !hit; ++q) {
        int64_t v[3], qq = q;
        for (int a = 0; a < d; ++a) {
          v[a] = r[a] - m + qq % span;
          qq /= span;
        }
        hit = flag_of(fctx, f, v);
      }
      if (!hit) break;
      --m;
    }
    if (st) st->order_hist[m]++;
    if (order_out) order_out[f] = (int8_t)m;
    /* Tensor-product sum of eq. "multiZ" over the (2m+2)^d stencil. */
    double w[3][6];
    for (int a = 0; a < d; ++a) orc_weights(m, xi[a], w[a]);
    int span = 2 * m + 2;
    double sum = 0.0;
    if (d == 2) {
      for (int ky = 0; ky < span; ++ky)
        for (int kx = 0; kx < span; ++kx) {
          int64_t v[3] = {r[0] - m + kx, r[1] - m + ky, 0};
          sum += fin[f][flatten_wrapped(P, v)] * w[0][kx] * w[1][ky];
        }
    } else if (d == 3) {
      for (int kz = 0; kz < span; ++kz)
        for (int ky = 0; ky < span; ++ky)
          for (int kx = 0; kx < span; ++kx) {
            int64_t v[3] = {r[0] - m + kx, r[1] - m + ky, r[2] - m + kz};
            sum += fin[f][flatten_wrapped(P, v)] * w[0][kx] * w[1][ky] * w[2][kz];
          }
    } else {
      for (int kx = 0; kx < span; ++kx) {
        int64_t v[3] = {r[0] - m + kx, 0, 0};
        sum += fin[f][flatten_wrapped(P, v)] * w[0][kx];
      }
    }
    out[f] = sum;
  }
  return ORC_OK;
}

typedef struct {
  const orc_problem *P;
  const uint8_t *flags;
} flagarr_ctx;

static int flag_from_array(void *vctx, int f, const int64_t *node) {
  flagarr_ctx *c = (flagarr_ctx *)vctx;
  return (c->flags[flatten_wrapped(c->P, node)] >> f) & 1;
}

typedef struct {
  const orc_problem *P;
  const double *const *fin;
} flagfly_ctx;

static int flag_on_demand(void *vctx, int f, const int64_t *node) {
  flagfly_ctx *c = (flagfly_ctx *)vctx;
  return orc_flag(c->P, c->fin[f], node);
}

static int check_problem(const orc_problem *P) {
  if (P->dim < 1 || P->dim > ORC_MAX_DIM) return ORC_EINVAL;
  if (P->nfields < 1 || P->nfields > ORC_MAX_FIELDS) return ORC_EINVAL;
  if (P->order_max < 0 || P->order_max > 2) return ORC_EINVAL;
  for (int a = 0; a < P->dim; ++a)
    if (P->n[a] < 2 * P->order_max + 2 || !(P->len[a] > 0.0)) return ORC_EINVAL;
  if (P->vel_kind == ORC_VEL_CARRIED && P->nfields < P->dim) return ORC_EINVAL;
  return ORC_OK;
}

/* Reconstruct every mesh node from the stored lattice displacement. */
/* orders, when not NULL, receives the order used per field and node
 * (nfields x Ntot, -1 where the search failed).                            */
int orc_reconstruct(const orc_problem *P, const double *disp,
                    const double *const *fin, double *const *fout,
                    orc_stats *stats, int8_t *orders) {
  if (check_problem(P) != ORC_OK) return ORC_EINVAL;
  int64_t N = total_nodes(P);
  uint8_t *flags = (uint8_t *)calloc((size_t)N, 1);
  if (!flags) return ORC_EINVAL;
  if (P->limiter) orc_flags(P, fin, flags);
  orc_stats tot;
  memset(&tot, 0, sizeof(tot));
  int first_err = ORC_OK;
#pragma omp parallel
  {
    orc_stats st;
    memset(&st, 0, sizeof(st));
    int err = ORC_OK;
    array_ctx dc = {P, disp, N};
    flagarr_ctx fc = {P, flags};
#pragma omp for schedule(static)
    for (int64_t lin = 0; lin < N; ++lin) {
      int64_t idx[3] = {0, 0, 0};
      double out[ORC_MAX_FIELDS];
      int8_t ord[ORC_MAX_FIELDS];
      unflatten(P, lin, idx);
      int rc = node_reconstruct(P, disp_from_array, &dc, flag_from_array, &fc,
                                fin, idx, out, ord, &st);
      if (rc != ORC_OK && err == ORC_OK) err = rc;
      for (int f = 0; f < P->nfields; ++f) {
        fout[f][lin] = out[f];
        if (orders) orders[f * N + lin] = ord[f];
      }
    }
#pragma omp critical
    {
      tot.search_fail += st.search_fail;
      tot.newton_fail += st.newton_fail;
      for (int m = 0; m < 3; ++m) tot.order_hist[m] += st.order_hist[m];
      tot.walk_steps += st.walk_steps;
      tot.newton_iters += st.newton_iters;
      if (err != ORC_OK && first_err == ORC_OK) first_err = err;
    }
  }
  tot.nodes = N;
  if (P->limiter)
    for (int64_t lin = 0; lin < N; ++lin)
      for (int f = 0; f < P->nfields; ++f) tot.flagged += (flags[lin] >> f) & 1;
  free(flags);
  if (stats) *stats = tot;
  return first_err;
}

/* One full step for a list of mesh nodes, with trajectories integrated on
 * demand for every lattice point the search touches (ksteps sub-steps of dt
 * from t before the reconstruction) and flags evaluated on demand.  Meant for
 * spot checks of large grids; out is count x nfields.                        */
int orc_step_sampled(const orc_problem *P, double t, double dt, int ksteps,
                     const double *const *fin, const int64_t *nodes,
                     int64_t count, double *out, orc_stats *stats) {
  if (check_problem(P) != ORC_OK || ksteps < 1) return ORC_EINVAL;
  orc_stats tot;
  memset(&tot, 0, sizeof(tot));
  int first_err = ORC_OK;
#pragma omp parallel
  {
    orc_stats st;
    memset(&st, 0, sizeof(st));
    int err = ORC_OK;
    /* A carried velocity is the fields themselves. */
    orc_problem Q = *P;
    if (P->vel_kind == ORC_VEL_CARRIED)
      for (int a = 0; a < P->dim; ++a) Q.ugrid[a] = fin[a];
    traj_ctx tc = {&Q, t, dt, ksteps};
    flagfly_ctx fc = {P, fin};
#pragma omp for schedule(dynamic, 16)
    for (int64_t s = 0; s < count; ++s) {
      int64_t idx[3] = {0, 0, 0};
      unflatten(P, nodes[s], idx);
      int rc = node_reconstruct(P, disp_on_demand, &tc,
                                P->limiter ? flag_on_demand : NULL, &fc, fin,
                                idx, out + s * P->nfields, NULL, &st);
      if (rc != ORC_OK && err == ORC_OK) err = rc;
    }
#pragma omp critical
    {
      tot.search_fail += st.search_fail;
      tot.newton_fail += st.newton_fail;
      for (int m = 0; m < 3; ++m) tot.order_hist[m] += st.order_hist[m];
      tot.walk_steps += st.walk_steps;
      tot.newton_iters += st.newton_iters;
      if (err != ORC_OK && first_err == ORC_OK) first_err = err;
    }
  }
  tot.nodes = count;
  if (stats) *stats = tot;
  return first_err;
}

static void accumulate_stats(orc_stats *tot, const orc_stats *st) {
  tot->nodes += st->nodes;
  tot->search_fail += st->search_fail;
  tot->newton_fail += st->newton_fail;
  for (int m = 0; m < 3; ++m) tot->order_hist[m] += st->order_hist[m];
  tot->flagged += st->flagged;
  tot->walk_steps += st->walk_steps;
  tot->newton_iters += st->newton_iters;
}

/* nsteps full steps, fields updated in place.  Each cycle resets the lattice,
 * integrates its trajectories over kevery sub-steps of dt and reconstructs the
 * fields on the mesh (Sec. 2: the lattice moves for a number of steps and is
 * then interpolated back and reset).  Step s covers [t0+s dt, t0+(s+1) dt];
 * nsteps must be a multiple of kevery.                                       */
static int run_cycles(const orc_problem *P, double t0, double dt, int nsteps, int kevery,
                      int store_f32, double *const *fields, orc_stats *stats);

int orc_run(const orc_problem *P, double t0, double dt, int nsteps, int kevery,
            double *const *fields, orc_stats *stats) {
  return run_cycles(P, t0, dt, nsteps, kevery, 0, fields, stats);
}

/* As orc_run, but every reconstructed value is rounded to the nearest FP32
 * number before the next cycle uses it: the values a run that stores its
 * fields in single precision carries from step to step (the FP32-value form,
 * whose positions, search and Newton stay FP64).  All arithmetic within a
 * step is still FP64.                                                        */
int orc_run_f32store(const orc_problem *P, double t0, double dt, int nsteps, int kevery,
                     double *const *fields, orc_stats *stats) {
  return run_cycles(P, t0, dt, nsteps, kevery, 1, fields, stats);
}

static int run_cycles(const orc_problem *P, double t0, double dt, int nsteps, int kevery,
                      int store_f32, double *const *fields, orc_stats *stats) {
  if (check_problem(P) != ORC_OK || kevery < 1 || nsteps % kevery != 0)
    return ORC_EINVAL;
  int64_t N = total_nodes(P);
  int nf = P->nfields;
  double *disp = (double *)malloc(sizeof(double) * (size_t)(N * P->dim));
  double *buf = (double *)malloc(sizeof(double) * (size_t)(N * nf));
  if (!disp || !buf) {
    free(disp);
    free(buf);
    return ORC_EINVAL;
  }
  double *outp[ORC_MAX_FIELDS];
  for (int f = 0; f < nf; ++f) outp[f] = buf + f * N;
  orc_stats tot;
  memset(&tot, 0, sizeof(tot));
  int rc = ORC_OK;
  /* A carried velocity is the fields at each reset. */
  orc_problem Q = *P;
  if (P->vel_kind == ORC_VEL_CARRIED)
    for (int a = 0; a < P->dim; ++a) Q.ugrid[a] = fields[a];
  for (int s = 0; s < nsteps && rc == ORC_OK; s += kevery) {
    memset(disp, 0, sizeof(double) * (size_t)(N * P->dim));
    for (int k = 0; k < kevery; ++k) orc_trajectories(&Q, t0 + (s + k) * dt, dt, disp);
    orc_stats st;
    rc = orc_reconstruct(P, disp, (const double *const *)fields, outp, &st, NULL);
    for (int f = 0; f < nf; ++f) memcpy(fields[f], outp[f], sizeof(double) * (size_t)N);
    if (store_f32)
      for (int f = 0; f < nf; ++f)
        for (int64_t i = 0; i < N; ++i) fields[f][i] = (double)(float)fields[f][i];
    accumulate_stats(&tot, &st);
  }
  free(disp);
  free(buf);
  if (stats) *stats = tot;
  return rc;
}

/* ------------------------------------------------------------------------- */
/* Source terms (Sec. 2: the right-hand side S_i of eq. "momento" may hold
 * spatial derivatives, taken by finite differences on the reference mesh).   */

/* Centred finite-difference weights c[0..2M] (offsets -M..M) of the p-th
 * derivative on a unit grid: the unique weights for which the rule is exact on
 * every polynomial of degree <= 2M, i.e. sum_k c_k k^q = q! [q == p] for
 * q = 0..2M.  Solved by Gaussian elimination with partial pivoting in long
 * double.  These are the "Taylor series from 2m+1 points" derivatives that the
 * cardinal Z-splines match at their knots (eq. "matchder").                   */
int orc_fd_weights(int M, int p, double *c) {
  if (M < 1 || M > 3 || p < 0 || p > 2 * M) return ORC_EINVAL;
  const int n = 2 * M + 1;
  long double A[7][8];
  for (int q = 0; q < n; ++q) {
    for (int j = 0; j < n; ++j) {
      long double k = (long double)(j - M), v = 1.0L;
      for (int e = 0; e < q; ++e) v *= k;
      A[q][j] = v;                       /* row q: k^q over the offsets */
    }
    long double fact = 1.0L;
    for (int e = 2; e <= q; ++e) fact *= (long double)e;
    A[q][n] = q == p ? fact : 0.0L;
  }
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (fabsl(A[r][col]) > fabsl(A[piv][col])) piv = r;
    if (A[piv][col] == 0.0L) return ORC_EINVAL;
    if (piv != col)
      for (int j = 0; j <= n; ++j) {
        long double t = A[col][j];
        A[col][j] = A[piv][j];
        A[piv][j] = t;
      }
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      long double f = A[r][col] / A[col][col];
      for (int j = col; j <= n; ++j) A[r][j] -= f * A[col][j];
    }
  }
  for (int j = 0; j < n; ++j) c[j] = (double)(A[j][n] / A[j][j]);
  return ORC_OK;
}

/* Half-width of the finite-difference rules: the 2m+1 points of the Z-spline
 * order in use, at least three points (Z0 matches no derivative).           */
static int fd_half_width(const orc_problem *P) {
  return P->order_max < 1 ? 1 : P->order_max;
}

/* Value of mesh field g at (i + di, j + dj), periodic (2-D). */
static double at2(const orc_problem *P, const double *g, int64_t i, int64_t j,
                  int di, int dj) {
  return g[orc_wrap(i + di, P->n[0]) + P->n[0] * orc_wrap(j + dj, P->n[1])];
}

/* Right-hand side of the shallow-water system, eq. "nlsw", at every mesh node
 * (2-D).  Fields: G[0] = u1, G[1] = u2 (the carried velocity), G[2] = h; any
 * further field is passive (no source).  With f = fc + beta (y - y0) and the
 * orthogonal velocity (-u2, u1):
 *   S_h  = -(1 + h) div u
 *   S_u1 = -dh/dx1 + f u2 + nu V1
 *   S_u2 = -dh/dx2 - f u1 + nu V2
 * where V = div[(1 + h)(grad u + grad u^T)], written out as
 *   V_i = (1 + h)(lap u_i + d_i div u) + sum_j (d_j h)(d_j u_i + d_i u_j).
 * Pure derivatives use the centred (2M+1)-point rules along one axis, mixed
 * ones the product of the two first-derivative rules.  The paper's equatorial
 * beta plane is fc = 0, beta = f0, y0 the equator.                           */
int orc_source_mesh(const orc_problem *P, const double *const *G, double *const *S) {
  if (P->dim != 2 || P->nfields < 3 || P->src_kind != ORC_SRC_SHALLOW_WATER)
    return ORC_EINVAL;
  const int M = fd_half_width(P);
  double c1[7], c2[7];
  if (orc_fd_weights(M, 1, c1) != ORC_OK || orc_fd_weights(M, 2, c2) != ORC_OK)
    return ORC_EINVAL;
  const double hx = P->len[0] / (double)P->n[0], hy = P->len[1] / (double)P->n[1];
  const double fc = P->sp[0], beta = P->sp[1], y0 = P->sp[2], nu = P->sp[3];
  const int64_t N = total_nodes(P);
#pragma omp parallel for schedule(static)
  for (int64_t lin = 0; lin < N; ++lin) {
    const int64_t i = lin % P->n[0], j = lin / P->n[0];
    double d1x[3] = {0, 0, 0}, d1y[3] = {0, 0, 0};
    double d2x[3] = {0, 0, 0}, d2y[3] = {0, 0, 0}, dxy[3] = {0, 0, 0};
    for (int c = 0; c < 3; ++c) {
      for (int k = -M; k <= M; ++k) {
        d1x[c] += c1[k + M] * at2(P, G[c], i, j, k, 0);
        d1y[c] += c1[k + M] * at2(P, G[c], i, j, 0, k);
        d2x[c] += c2[k + M] * at2(P, G[c], i, j, k, 0);
        d2y[c] += c2[k + M] * at2(P, G[c], i, j, 0, k);
      }
      for (int b = -M; b <= M; ++b)
        for (int a = -M; a <= M; ++a)
          dxy[c] += c1[a + M] * c1[b + M] * at2(P, G[c], i, j, a, b);
      d1x[c] /= hx;
      d1y[c] /= hy;
      d2x[c] /= hx * hx;
      d2y[c] /= hy * hy;
      dxy[c] /= hx * hy;
    }
    const double u = G[0][lin], v = G[1][lin], h = G[2][lin];
    const double f = fc + beta * ((double)j * hy - y0);
    const double div = d1x[0] + d1y[1];
    double su = -d1x[2] + f * v;
    double sv = -d1y[2] - f * u;
    const double sh = -(1.0 + h) * div;
    if (nu != 0.0) {
      /* V_1 = (1+h)(u_xx + u_yy + u_xx + v_xy) + h_x (2 u_x) + h_y (u_y + v_x)
       * V_2 = (1+h)(v_xx + v_yy + u_xy + v_yy) + h_x (v_x + u_y) + h_y (2 v_y) */
      const double V1 = (1.0 + h) * (d2x[0] + d2y[0] + d2x[0] + dxy[1]) +
                        d1x[2] * (d1x[0] + d1x[0]) + d1y[2] * (d1y[0] + d1x[1]);
      const double V2 = (1.0 + h) * (d2x[1] + d2y[1] + dxy[0] + d2y[1]) +
                        d1x[2] * (d1x[1] + d1y[0]) + d1y[2] * (d1y[1] + d1y[1]);
      su += nu * V1;
      sv += nu * V2;
    }
    S[0][lin] = su;
    S[1][lin] = sv;
    S[2][lin] = sh;
  }
  return ORC_OK;
}

/* nsteps steps of a system with source terms (2-D shallow water, carried
 * velocity), lattice reset every step.  Within the step [t, t+dt] every
 * lattice node carries its position X and its values H, integrated with the
 * low-storage third-order Runge-Kutta of Williamson (Sec. 2):
 *   stage s = 0, 1, 2:
 *     G   = the stage fields on the mesh: the fields at t for s = 0, else the
 *           reconstruction (Sec. 2.1-2.3) of the lattice values H at X;
 *     S   = the right-hand side on the mesh from G (orc_source_mesh);
 *     per lattice node:  u = its own velocity H[0..1],
 *                        s_hat = S interpolated at X (Z-spline, order_max),
 *       qX = A_s qX + dt u,      X += B_s qX,
 *       qH = A_s qH + dt s_hat,  H += B_s qH   (fields 0..2; others passive);
 *   then the fields at t+dt are the reconstruction of H at X (the reset).
 * Stats accumulate over all three reconstructions of each step.             */
int orc_run_source(const orc_problem *P, double t0, double dt, int nsteps,
                   double *const *fields, orc_stats *stats) {
  if (check_problem(P) != ORC_OK || P->dim != 2 || P->nfields < 3 ||
      P->src_kind != ORC_SRC_SHALLOW_WATER || P->vel_kind != ORC_VEL_CARRIED ||
      nsteps < 0)
    return ORC_EINVAL;
  static const double A[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
  static const double B[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};
  (void)t0;  /* the shallow-water source does not depend on t explicitly */
  const int64_t N = total_nodes(P);
  const int nf = P->nfields;
  double *disp = (double *)calloc((size_t)(2 * N), sizeof(double));
  double *qx = (double *)calloc((size_t)(2 * N), sizeof(double));
  double *H = (double *)calloc((size_t)(nf * N), sizeof(double));
  double *qh = (double *)calloc((size_t)(3 * N), sizeof(double));
  double *G = (double *)calloc((size_t)(nf * N), sizeof(double));
  double *S = (double *)calloc((size_t)(3 * N), sizeof(double));
  int rc = ORC_OK;
  if (!disp || !qx || !H || !qh || !G || !S) rc = ORC_EINVAL;
  double *Hp[ORC_MAX_FIELDS], *Gp[ORC_MAX_FIELDS], *Sp[3];
  for (int f = 0; f < nf; ++f) {
    Hp[f] = H ? H + f * N : NULL;
    Gp[f] = G ? G + f * N : NULL;
  }
  for (int c = 0; c < 3; ++c) Sp[c] = S ? S + c * N : NULL;
  const double hx[2] = {P->len[0] / (double)P->n[0], P->len[1] / (double)P->n[1]};
  orc_stats tot;
  memset(&tot, 0, sizeof(tot));
  for (int step = 0; step < nsteps && rc == ORC_OK; ++step) {
    for (int f = 0; f < nf; ++f) memcpy(Hp[f], fields[f], sizeof(double) * (size_t)N);
    memset(disp, 0, sizeof(double) * (size_t)(2 * N));
    memset(qx, 0, sizeof(double) * (size_t)(2 * N));
    memset(qh, 0, sizeof(double) * (size_t)(3 * N));
    for (int s = 0; s < 3 && rc == ORC_OK; ++s) {
      const double *const *Gs = (const double *const *)fields;
      if (s > 0) {
        orc_stats st;
        rc = orc_reconstruct(P, disp, (const double *const *)Hp, Gp, &st, NULL);
        accumulate_stats(&tot, &st);
        Gs = (const double *const *)Gp;
      }
      if (rc == ORC_OK) rc = orc_source_mesh(P, Gs, Sp);
      if (rc != ORC_OK) break;
#pragma omp parallel for schedule(static)
      for (int64_t lin = 0; lin < N; ++lin) {
        const int64_t idx[2] = {lin % P->n[0], lin / P->n[0]};
        double x[3] = {0.0, 0.0, 0.0}, sh[3];
        for (int a = 0; a < 2; ++a) x[a] = ((double)idx[a] + disp[a * N + lin]) * hx[a];
        orc_zinterp(P, P->order_max, 3, (const double *const *)Sp, x, sh);
        for (int a = 0; a < 2; ++a) {
          const double ua = Hp[a][lin];
          qx[a * N + lin] = A[s] * qx[a * N + lin] + dt * ua / hx[a];
          disp[a * N + lin] += B[s] * qx[a * N + lin];
        }
        for (int c = 0; c < 3; ++c) {
          qh[c * N + lin] = A[s] * qh[c * N + lin] + dt * sh[c];
          Hp[c][lin] += B[s] * qh[c * N + lin];
        }
      }
    }
    if (rc != ORC_OK) break;
    orc_stats st;
    rc = orc_reconstruct(P, disp, (const double *const *)Hp, (double *const *)fields, &st,
                         NULL);
    accumulate_stats(&tot, &st);
  }
  free(disp);
  free(qx);
  free(H);
  free(qh);
  free(G);
  free(S);
  if (stats) *stats = tot;
  return rc;
}

/* Number of OpenMP threads the oracle's parallel loops use. */
int orc_threads(void) { return omp_get_max_threads(); }
