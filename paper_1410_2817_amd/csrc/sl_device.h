// Device building blocks of the forward semi-Lagrangian step for gfx950:
// prescribed velocities, cardinal Z-spline weights, the element map inversion
// and the host-element search.  Everything here is header-only so that the
// kernels in sl.hip inline it.
#pragma once

#include <hip/hip_runtime.h>
#include <limits.h>
#include <stdint.h>

#include "sl.h"

namespace sl {

// ---------------------------------------------------------------------------
// Kernel argument blocks (passed by value; they live in the kernarg segment).

struct GridArgs {
  int n[3];
  int ntot;
  double h[3];
  double rh[3];   // 1 / h_a, correctly rounded (host)
  double r6h[3];  // 1 / (6 h_a), correctly rounded (host)
  int nfields;
  int order_max;
  int limiter;
  double theta;
  int newton_max_iter;
  double newton_tol;
  int walk_max;
  int scan_radius;
  double eps;
  int off[3];  // index of node 0 in the whole lattice (a shard); 0 otherwise
};

// Fourier mode q adds amp * cos(theta) to the velocity, theta = pi k . y +
// phase with y_a = 2 x_a / L_a.  Two encodings, one per grid
// (VelArgs::small_k):
//   gen: any wave vector; theta / pi = phase / pi + c . x (c_a = 2 k_a / L_a),
//        one cospi per mode and point;
//   ik:  2-D integer wave vectors with |k_a| <= kSmallK; e^{i theta} = e^{i phase}
//        prod_a (e^{i pi y_a})^{k_a}, from e^{i pi y_a}, which all modes share
//        (sum_a |k_a| complex products per mode instead of a cosine).
constexpr int kSmallK = 4;

struct Mode {
  double amp[3];
  union {
    struct {
      double c[3];
      double phase_over_pi;
    } gen;
    struct {
      double cphi, sphi;  // cos and sin of the phase
      int k[3];
      int unused;
    } ik;
  };
  double pad;
};

struct VelArgs {
  int kind;
  int nmodes;
  int small_k;        // SL_VEL_FOURIER: modes in the ik encoding
  double kscale[3];   // SL_VEL_FOURIER: 2 / L_a (y_a = kscale_a x_a)
  // Bound on |delta| / dt over the Runge-Kutta stage offsets delta that the
  // angle-shift evaluators (NodeVelocity) take, in the units of their sincospi
  // argument, for the grid's family and integrator; 0 if none is known.
  double shift_rate;
  double p[8];
  Mode mode[SL_MAX_MODES];
  // SL_VEL_GRIDDED: samples on the mesh (x first), mesh spacing and size,
  // interpolation order.
  const double* ug[3];
  double ug_h[3];
  int ug_n[3];
  int ug_m;
};

struct FieldPtrs {
  const void* in[SL_MAX_FIELDS];
  void* out[SL_MAX_FIELDS];
};

// Slots of the device counter block at the start of the workspace.
enum StatSlot {
  ST_NODES = 0,
  ST_SEARCH_FAIL,
  ST_NEWTON_FAIL,
  ST_NONFINITE,
  ST_ORDER0,
  ST_ORDER1,
  ST_ORDER2,
  ST_WALKED,
  ST_SCANNED,
  ST_COUNT
};

// The counter block holds kStatCopies copies of the ST_COUNT counters, each
// on a 128-byte line of its own.  A workgroup adds its sums into copy
// blockIdx % kStatCopies: one copy per workgroup and counter would otherwise
// queue every workgroup's atomics on one L2 line.  Consecutive workgroups go
// to the 8 XCDs in turn, so each copy is only touched from one XCD.  The host
// adds the copies up when it reads the counters.
constexpr int kStatCopies = 64;
constexpr int kStatStride = 16;  // counters per copy: one 128-byte line
constexpr int kStatWords = kStatCopies * kStatStride;
static_assert(ST_COUNT <= kStatStride, "counter copy overflows its line");

__device__ __forceinline__ unsigned long long* stat_copy(unsigned long long* stats) {
  return stats + (blockIdx.x % kStatCopies) * kStatStride;
}

// Host: the totals of the copies (copies: kStatWords words, out: ST_COUNT).
inline void stat_totals(const unsigned long long* copies, unsigned long long* out) {
  for (int k = 0; k < ST_COUNT; ++k) out[k] = 0ull;
  for (int c = 0; c < kStatCopies; ++c)
    for (int k = 0; k < ST_COUNT; ++k) out[k] += copies[c * kStatStride + k];
}

__device__ __forceinline__ int wrap_index(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

// Wrap an index known to lie near [0, n) without integer division; far
// indices (only from pathological walks) take the general path.
__device__ __forceinline__ int wrap_near(int v, int n) {
  v = v < 0 ? v + n : v;
  v = v >= n ? v - n : v;
  return (unsigned)v < (unsigned)n ? v : wrap_index(v, n);
}

// Butterfly reductions over the 64 lanes of a wave (all lanes active).
// Wave-wide reductions over the 64 lanes with DPP lane moves (all lanes must
// be active): two quad exchanges, the half-row and row mirrors reduce each
// row of 16, then the broadcasts of lanes 15 and 31 into the following rows
// gather the whole wave in lane 63, which is read out as a wave-uniform
// value.  Each step is one VALU instruction with no LDS round trip (a
// butterfly of shuffles went through ds_bpermute and waited on LDS at every
// step).
template <class Op>
__device__ __forceinline__ int wave_reduce(int v, int identity, Op op) {
  v = op(v, __builtin_amdgcn_mov_dpp(v, 0xb1, 0xf, 0xf, false));   // quad_perm 1,0,3,2
  v = op(v, __builtin_amdgcn_mov_dpp(v, 0x4e, 0xf, 0xf, false));   // quad_perm 2,3,0,1
  v = op(v, __builtin_amdgcn_mov_dpp(v, 0x141, 0xf, 0xf, false));  // row_half_mirror
  v = op(v, __builtin_amdgcn_mov_dpp(v, 0x140, 0xf, 0xf, false));  // row_mirror
  v = op(v, __builtin_amdgcn_update_dpp(identity, v, 0x142, 0xa, 0xf, false));  // row_bcast:15
  v = op(v, __builtin_amdgcn_update_dpp(identity, v, 0x143, 0xc, 0xf, false));  // row_bcast:31
  return __builtin_amdgcn_readlane(v, 63);
}

__device__ __forceinline__ int wave_min(int v) {
  return wave_reduce(v, INT_MAX, [](int a, int b) { return min(a, b); });
}

__device__ __forceinline__ int wave_max(int v) {
  return wave_reduce(v, INT_MIN, [](int a, int b) { return max(a, b); });
}

__device__ __forceinline__ unsigned wave_sum(unsigned v) {
  return (unsigned)wave_reduce((int)v, 0, [](int a, int b) { return (int)((unsigned)a + (unsigned)b); });
}

// Adds the number of active lanes with `pred` to *ctr, one atomic per wave and
// only when the count is non-zero.  Must be reached by all active lanes.
__device__ __forceinline__ void wave_count(unsigned long long* ctr, bool pred) {
  unsigned long long m = __ballot(pred);
  if (m) {
    unsigned long long act = __ballot(1);
    if ((int)__lane_id() == __ffsll((long long)act) - 1)
      atomicAdd(ctr, (unsigned long long)__popcll(m));
  }
}

// ---------------------------------------------------------------------------
// Prescribed velocity u(x, t) (physical units).  `tf` is the time factor
// cos(pi t / p0) of the periodic families, evaluated once per stage.

// Tab (FP64 only): Z2 coefficients from constant memory (kZ2Coef) rather
// than literals.
template <typename T, bool Tab = true>
__device__ __forceinline__ void zspline_weights(int m, T t, T* w);

// cos(pi x) for the general Fourier encoding.  With n the integer nearest x
// and t = x - n (both exact), cos(pi x) = (-1)^n cos(pi t), |t| <= 1/2, and
// cos(pi t) = 1 + s P(s), s = t^2, with P the degree-7 Chebyshev interpolant
// of (cos(pi sqrt(s)) - 1) / s on [0, 1/4] (interpolation error below 1e-20;
// absolute error of the evaluation about 2e-16).  Coefficients, constant term
// first, from csrc/cospi_poly.py.  The library cospi's general argument
// handling cost about twice the instructions per mode, and the Taylor series
// in pi t it replaced took four more.  Tab: from constant memory (scalar
// operands of the FMAs); otherwise literals, which the mode loop keeps in
// vector registers.  The 2-D kernels embed every velocity family and spill
// the scalar registers the table takes, so only 3-D grids use it.  Not
// static, for the reason given at kTaylorSinCos.
__constant__ double kCosPiPoly[8] = {
    -4.934802200544679,    4.058712126416736,      -1.3352627688518803,
    0.2353306302721577,    -0.02580689002587539,   0.001929562652479866,
    -0.00010458286368326585, 4.166399462726949e-06};

template <bool Tab>
__device__ __forceinline__ double cospi_poly(double x) {
  const double n = rint(x);
  const double t = x - n;
  const double s = t * t;
  double p;
  if constexpr (Tab) {
    const double* k = kCosPiPoly;
    p = k[7];
#pragma unroll
    for (int i = 6; i >= 0; --i) p = fma(p, s, k[i]);
  } else {
    p = 4.166399462726949e-06;
    p = fma(p, s, -0.00010458286368326585);
    p = fma(p, s, 0.001929562652479866);
    p = fma(p, s, -0.02580689002587539);
    p = fma(p, s, 0.2353306302721577);
    p = fma(p, s, -1.3352627688518803);
    p = fma(p, s, 4.058712126416736);
    p = fma(p, s, -4.934802200544679);
  }
  p = fma(p, s, 1.0);
  const double h = 0.5 * n;
  return h != rint(h) ? -p : p;
}

// Sum of the modes in the ik encoding at the point with sin/cos(pi y_a) =
// sn[a] / cs[a]: e^{i theta} = e^{i phase} times |k_a| factors e^{+-i pi y_a}
// per axis.  The wave vectors are wave-uniform, so these are scalar loops
// (a branch per power would be if-converted into selects over every power).
template <int D>
__device__ __forceinline__ void fourier_small_k(const VelArgs& v, const double* sn,
                                                const double* cs, double* u) {
#pragma unroll
  for (int a = 0; a < D; ++a) u[a] = 0.0;
  for (int q = 0; q < v.nmodes; ++q) {
    const Mode& md = v.mode[q];
    double zr = md.ik.cphi, zi = md.ik.sphi;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int k = md.ik.k[a];
      const double r = cs[a], s = k < 0 ? -sn[a] : sn[a];
#pragma unroll 1
      for (int j = k < 0 ? -k : k; j > 0; --j) {
        const double t = zr * r - zi * s;
        zi = zr * s + zi * r;
        zr = t;
      }
    }
#pragma unroll
    for (int a = 0; a < D; ++a) u[a] = fma(md.amp[a], zr, u[a]);
  }
}

template <int VK, int D>
__device__ __forceinline__ void velocity(const VelArgs& v, const double* x, double tf,
                                         double* u) {
  if constexpr (VK == SL_VEL_UNIFORM) {
    for (int a = 0; a < D; ++a) u[a] = v.p[a];
  } else if constexpr (VK == SL_VEL_SOLID_BODY) {
    u[0] = -v.p[0] * (x[1] - v.p[2]);
    u[1] = v.p[0] * (x[0] - v.p[1]);
    if constexpr (D == 3) u[2] = 0.0;
  } else if constexpr (VK == SL_VEL_SWIRL2D) {
    double sx, cx, sy, cy;
    sincospi(x[0], &sx, &cx);
    sincospi(x[1], &sy, &cy);
    const double s = v.p[1] * tf;
    // sin(2 pi y) = 2 sin(pi y) cos(pi y)
    u[0] = s * sx * sx * (2.0 * sy * cy);
    u[1] = -s * sy * sy * (2.0 * sx * cx);
    if constexpr (D == 3) u[2] = 0.0;
  } else if constexpr (VK == SL_VEL_DEFORM3D && D == 3) {
    double sx, cx, sy, cy, sz, cz;
    sincospi(x[0], &sx, &cx);
    sincospi(x[1], &sy, &cy);
    sincospi(x[2], &sz, &cz);
    const double s = v.p[1] * tf;
    const double s2x = 2.0 * sx * cx, s2y = 2.0 * sy * cy, s2z = 2.0 * sz * cz;
    u[0] = 2.0 * s * sx * sx * s2y * s2z;
    u[1] = -s * s2x * sy * sy * s2z;
    u[2] = -s * s2x * s2y * sz * sz;
  } else if constexpr (VK == SL_VEL_FOURIER) {
    if (v.small_k) {
      double sn[D], cs[D];
#pragma unroll
      for (int a = 0; a < D; ++a) sincospi(x[a] * v.kscale[a], &sn[a], &cs[a]);
      fourier_small_k<D>(v, sn, cs, u);
      return;
    }
    for (int a = 0; a < D; ++a) u[a] = 0.0;
    for (int q = 0; q < v.nmodes; ++q) {
      const Mode& md = v.mode[q];
      double th = md.gen.phase_over_pi;
      for (int a = 0; a < D; ++a) th += md.gen.c[a] * x[a];
      const double cs = cospi_poly<D == 3>(th);
      for (int a = 0; a < D; ++a) u[a] += md.amp[a] * cs;
    }
  } else if constexpr (VK == SL_VEL_GRIDDED) {
    // Tensor-product Z-spline interpolation of the mesh samples (eq. "multiZ"
    // applied to the velocity), periodic; slot k holds node r - 2 + k.
    int r[3] = {0, 0, 0};
    double w[3][6];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const double sa = x[a] / v.ug_h[a];
      r[a] = (int)floor(sa);
      zspline_weights<double>(v.ug_m, sa - (double)r[a], w[a]);
    }
#pragma unroll
    for (int a = 0; a < D; ++a) u[a] = 0.0;
    // Slots outside the order's window carry zero weight and are skipped
    // (wave-uniform tests on constant indices, so the weights stay in
    // registers).
    const int lo = 2 - v.ug_m, hi = 3 + v.ug_m;
    const int nx = v.ug_n[0], ny = v.ug_n[1];
#pragma unroll 1
    for (int kz = (D == 3 ? lo : 0); kz <= (D == 3 ? hi : 0); ++kz) {
      const int iz = D == 3 ? wrap_index(r[2] - 2 + kz, v.ug_n[2]) : 0;
      // Rolled loop: wz by selects (a dynamic index would go to scratch).
      double wz = 1.0;
      if (D == 3) {
        wz = w[2][5];
#pragma unroll
        for (int q = 4; q >= 0; --q) wz = kz == q ? w[2][q] : wz;
      }
#pragma unroll
      for (int ky = 0; ky < 6; ++ky) {
        if (ky < lo || ky > hi) continue;
        const int iy = wrap_index(r[1] - 2 + ky, ny);
        const int row = nx * (iy + ny * iz);
        double sx[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int kx = 0; kx < 6; ++kx) {
          if (kx < lo || kx > hi) continue;
          const int lin = row + wrap_index(r[0] - 2 + kx, nx);
#pragma unroll
          for (int a = 0; a < D; ++a) sx[a] = fma(v.ug[a][lin], w[0][kx], sx[a]);
        }
        const double wyz = w[1][ky] * wz;
#pragma unroll
        for (int a = 0; a < D; ++a) u[a] = fma(sx[a], wyz, u[a]);
      }
    }
  } else {
    // Combinations rejected at grid creation (a 3-D family on a 2-D grid).
    for (int a = 0; a < D; ++a) u[a] = 0.0;
  }
}

// a / b with y = RN(1 / b) given: q = RN(a y) corrected once by the exact
// remainder a - b q (an FMA), q + (a - b q) y, which is Markstein's
// correction step (P. Markstein, IBM J. Res. Dev. 34(1), 1990); for the
// moderate magnitudes here it returns the correctly rounded quotient, so a
// displacement of whole cells stays exact.  Three operations against the
// ten of a general division.
__device__ __forceinline__ double div_by(double a, double b, double y) {
  const double q = a * y;
  return fma(fma(-q, b, a), y, q);
}

// ---------------------------------------------------------------------------
// Velocity at the Runge-Kutta stage points of one lattice node.  The stage
// points are x0 + delta with delta a few cells at most, so the periodic
// families evaluate sin/cos(pi x0) once and reach each stage point by angle
// addition with sin/cos(pi delta) from short Taylor series; `tf` is the time
// factor cos(pi t / p0) of the stage, computed on the host.

// Taylor coefficients of sin (z, z^3, ..., z^9: [4] .. [0]) and cos (1, z^2,
// ..., z^10: [10] .. [5]).  Kept in constant memory, they reach the FMAs as
// scalar operands; as literals each 64-bit constant took two VALU moves.  Not
// static: with internal linkage the compiler folds them back into literals.
__constant__ double kTaylorSinCos[11] = {
    1.0 / 362880,   -1.0 / 5040,  1.0 / 120, -1.0 / 6, 1.0,  // sin
    -1.0 / 3628800, 1.0 / 40320, -1.0 / 720, 1.0 / 24, -0.5, 1.0};  // cos

// sin(pi d) and cos(pi d): Taylor series to z^9 / z^10 (z = pi d) for
// |d| <= 1/32, where the truncation error is below 2e-19; sincospi beyond.
__device__ __forceinline__ void sincospi_near0(double d, double* s, double* c) {
  if (fabs(d) <= 0.03125) {
    const double z = 3.141592653589793 * d, z2 = z * z;
    const double* k = kTaylorSinCos;
    *s = z * (k[4] + z2 * (k[3] + z2 * (k[2] + z2 * (k[1] + z2 * k[0]))));
    *c = k[10] + z2 * (k[9] + z2 * (k[8] + z2 * (k[7] + z2 * (k[6] + z2 * k[5]))));
  } else {
    sincospi(d, s, c);
  }
}

// The same for |d| <= kSmallShift (z <= 0.0246), with the series to z^7 / z^6:
// truncation below 1e-20 (sin) and 4e-18 (cos).
constexpr double kSmallShift = 1.0 / 128;
__device__ __forceinline__ void sincospi_small(double d, double* s, double* c) {
  const double z = 3.141592653589793 * d, z2 = z * z;
  const double* k = kTaylorSinCos;
  *s = z * (k[4] + z2 * (k[3] + z2 * (k[2] + z2 * k[1])));
  *c = k[10] + z2 * (k[9] + z2 * (k[8] + z2 * k[7]));
}

// sin/cos(pi (x0 + d)) from s0 = sin(pi x0), c0 = cos(pi x0).  `small`
// (wave-uniform): |d| <= kSmallShift is known for every stage offset.
__device__ __forceinline__ void sincospi_shift(double s0, double c0, double d, bool small,
                                               double* s, double* c) {
  double sd, cd;
  if (small)
    sincospi_small(d, &sd, &cd);
  else
    sincospi_near0(d, &sd, &cd);
  *s = s0 * cd + c0 * sd;
  *c = c0 * cd - s0 * sd;
}

template <int VK, int D>
struct NodeVelocity {
  double s0[3], c0[3];
  bool small;  // every stage offset within kSmallShift (wave-uniform)

  // From the per-axis table of trig_table_kernel (sl_traj.h) instead: the
  // same values at a lattice node that sits on its mesh node (x0 = idx h).
  __device__ __forceinline__ void init_table(const double* __restrict__ trig, const GridArgs& g,
                                             const int* idx, bool small_shift) {
    small = small_shift;
    if constexpr (VK == SL_VEL_SWIRL2D || (VK == SL_VEL_DEFORM3D && D == 3) ||
                  VK == SL_VEL_FOURIER) {
      constexpr int NA = VK == SL_VEL_SWIRL2D ? 2 : D;
      int base = 0;
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        s0[a] = trig[base + idx[a]];
        c0[a] = trig[base + g.n[a] + idx[a]];
        base += 2 * g.n[a];
      }
    }
  }

  // SL_VEL_FOURIER in the ik encoding: s0/c0 hold sin/cos(pi y_a) at x0.
  __device__ __forceinline__ void init(const VelArgs& v, const double* x0, bool small_shift) {
    small = small_shift;
    if constexpr (VK == SL_VEL_SWIRL2D || (VK == SL_VEL_DEFORM3D && D == 3)) {
      constexpr int NA = VK == SL_VEL_SWIRL2D ? 2 : 3;
#pragma unroll
      for (int a = 0; a < NA; ++a) sincospi(x0[a], &s0[a], &c0[a]);
    } else if constexpr (VK == SL_VEL_FOURIER) {
      if (v.small_k) {
#pragma unroll
        for (int a = 0; a < D; ++a) sincospi(x0[a] * v.kscale[a], &s0[a], &c0[a]);
      }
    }
  }

  // Velocity at x0 + delta (delta == nullptr: at x0 itself).
  __device__ __forceinline__ void eval(const VelArgs& v, const double* x0, const double* delta,
                                       double tf, double* u) const {
    if constexpr (VK == SL_VEL_SWIRL2D || (VK == SL_VEL_DEFORM3D && D == 3)) {
      constexpr int NA = VK == SL_VEL_SWIRL2D ? 2 : 3;
      double sn[3], cs[3];
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        if (delta) {
          sincospi_shift(s0[a], c0[a], delta[a], small, &sn[a], &cs[a]);
        } else {
          sn[a] = s0[a];
          cs[a] = c0[a];
        }
      }
      const double s = v.p[1] * tf;
      if constexpr (VK == SL_VEL_SWIRL2D) {
        // sin(2 pi y) = 2 sin(pi y) cos(pi y)
        u[0] = s * sn[0] * sn[0] * (2.0 * sn[1] * cs[1]);
        u[1] = -s * sn[1] * sn[1] * (2.0 * sn[0] * cs[0]);
        if constexpr (D == 3) u[2] = 0.0;
      } else {
        const double s2x = 2.0 * sn[0] * cs[0], s2y = 2.0 * sn[1] * cs[1],
                     s2z = 2.0 * sn[2] * cs[2];
        u[0] = 2.0 * s * sn[0] * sn[0] * s2y * s2z;
        u[1] = -s * s2x * sn[1] * sn[1] * s2z;
        u[2] = -s * s2x * s2y * sn[2] * sn[2];
      }
    } else {
      if constexpr (VK == SL_VEL_FOURIER) {
        if (v.small_k) {
          double sn[D], cs[D];
#pragma unroll
          for (int a = 0; a < D; ++a) {
            if (delta) {
              sincospi_shift(s0[a], c0[a], delta[a] * v.kscale[a], small, &sn[a], &cs[a]);
            } else {
              sn[a] = s0[a];
              cs[a] = c0[a];
            }
          }
          fourier_small_k<D>(v, sn, cs, u);
          return;
        }
      }
      double x[D];
#pragma unroll
      for (int a = 0; a < D; ++a) x[a] = delta ? x0[a] + delta[a] : x0[a];
      velocity<VK, D>(v, x, tf, u);
    }
  }
};

// ---------------------------------------------------------------------------
// Cardinal Z-spline weights (Appendix).  For a point r + t, slot s = k + 2
// holds the weight Z_m(t - k) of node r + k, k = -2..3; slots outside the
// order-m stencil are zero.

// The Z2 coefficients below as FP64, in the order they appear there.  The
// FP64 weights read them from constant memory so that the FMAs take them as
// scalar operands (as FP64 literals each took two VALU moves; FP32 literals
// fit the instructions).  Not static, for the reason given at kTaylorSinCos.
// The 2-D reconstruction kernels keep the literals (Tab = false): there the
// scalar registers the table takes are spilled.
__constant__ double kZ2Coef[28] = {
    1.0 / 12,  -1.0 / 24,  -3.0 / 8,   13.0 / 24,  -5.0 / 24,   // w0
    -2.0 / 3,  2.0 / 3,    13.0 / 8,   -8.0 / 3,   25.0 / 24,   // w1
    -5.0 / 4,  -35.0 / 12, 21.0 / 4,   -25.0 / 12,              // w2
    2.0 / 3,   2.0 / 3,    11.0 / 4,   -31.0 / 6,  25.0 / 12,   // w3
    -1.0 / 12, -1.0 / 24,  -11.0 / 8,  61.0 / 24,  -25.0 / 24,  // w4
    7.0 / 24,  -1.0 / 2,   5.0 / 24,   0.0};                    // w5

template <typename T, bool Tab>
__device__ __forceinline__ void zspline_weights(int m, T t, T* w) {
  // Each weight is its degree-(2m+1) polynomial in t in Horner form, with the
  // Appendix's rational coefficients; every weight but the node's own has no
  // constant term, so t = 0 gives exactly the unit weight on slot 2.
  const T one = T(1);
  const T t2 = t * t;
  if constexpr (sizeof(T) == 8 && Tab) {
    if (m == 2) {
      // The same polynomials as below, coefficients from kZ2Coef.
      const double* k = kZ2Coef;
      w[0] = t * (k[0] + t * (k[1] + t * (k[2] + t * (k[3] + t * k[4]))));
      w[1] = t * (k[5] + t * (k[6] + t * (k[7] + t * (k[8] + t * k[9]))));
      w[2] = one + t2 * (k[10] + t * (k[11] + t * (k[12] + t * k[13])));
      w[3] = t * (k[14] + t * (k[15] + t * (k[16] + t * (k[17] + t * k[18]))));
      w[4] = t * (k[19] + t * (k[20] + t * (k[21] + t * (k[22] + t * k[23]))));
      w[5] = t2 * t * (k[24] + t * (k[25] + t * k[26]));
      return;
    }
  }
  if (m == 2) {
    // Z2(t + 2) = -t (t-1)^3 (5t + 2) / 24
    w[0] = t * (T(1.0 / 12) + t * (T(-1.0 / 24) + t * (T(-3.0 / 8) + t * (T(13.0 / 24) + t * T(-5.0 / 24)))));
    // Z2(t + 1) = t (t-1) (25t^3 - 39t^2 + 16) / 24
    w[1] = t * (T(-2.0 / 3) + t * (T(2.0 / 3) + t * (T(13.0 / 8) + t * (T(-8.0 / 3) + t * T(25.0 / 24)))));
    // Z2(t) = -(t-1) (25t^4 - 38t^3 - 3t^2 + 12t + 12) / 12
    w[2] = one + t2 * (T(-5.0 / 4) + t * (T(-35.0 / 12) + t * (T(21.0 / 4) + t * T(-25.0 / 12))));
    // Z2(1 - t) = t (25t^4 - 62t^3 + 33t^2 + 8t + 8) / 12
    w[3] = t * (T(2.0 / 3) + t * (T(2.0 / 3) + t * (T(11.0 / 4) + t * (T(-31.0 / 6) + t * T(25.0 / 12)))));
    // Z2(2 - t) = -t (t-1) (25t^3 - 36t^2 - 3t - 2) / 24
    w[4] = t * (T(-1.0 / 12) + t * (T(-1.0 / 24) + t * (T(-11.0 / 8) + t * (T(61.0 / 24) + t * T(-25.0 / 24)))));
    // Z2(3 - t) = t^3 (t-1) (5t - 7) / 24
    w[5] = t2 * t * (T(7.0 / 24) + t * (T(-1.0 / 2) + t * T(5.0 / 24)));
  } else if (m == 1) {
    w[0] = T(0);
    // Z1(t + 1) = -t (t-1)^2 / 2
    w[1] = t * (T(-0.5) + t * (one + t * T(-0.5)));
    // Z1(t) = (t-1) (3t^2 - 2t - 2) / 2
    w[2] = one + t2 * (T(-2.5) + t * T(1.5));
    // Z1(1 - t) = -t (3t^2 - 4t - 1) / 2
    w[3] = t * (T(0.5) + t * (T(2) + t * T(-1.5)));
    // Z1(2 - t) = t^2 (t-1) / 2
    w[4] = t2 * (T(-0.5) + t * T(0.5));
    w[5] = T(0);
  } else {
    w[0] = T(0);
    w[1] = T(0);
    w[2] = one - t;
    w[3] = t;
    w[4] = T(0);
    w[5] = T(0);
  }
}

// ---------------------------------------------------------------------------
// Inversion of the multilinear (Z0) map of one deformed element (Sec. 2.2).
//
// V[e] = X(r + e) - x' are the element's vertex positions relative to the
// target mesh point, e in {0,1}^D with bit a for axis a.  Expanding the map
// about vertex r gives the finite series of eq. "mapping1":
//   F(xi) = V0 + sum_a A_a xi_a + sum_{a<b} B_ab xi_a xi_b (+ C xi_0 xi_1 xi_2).
// Newton's method solves F = 0 starting from the root of the linear part.
// solve() returns 1 if Newton converged (xi = solution), 0 if only the linear
// root is available (xi = that), -1 if the linear part is singular.
//
// Reciprocals are the hardware estimate refined by one Newton-Raphson step
// (exact for powers of two; the next Newton iteration absorbs any residual).
// The first kFastNewton iterations run unconditionally: Newton's, then chord
// iterations that keep its Jacobian (from the linear root each cuts the error
// by about the element's non-affine part times the first step, as fast as
// Newton's here at a third of the arithmetic in 3-D).  Lanes not converged
// after them continue with Newton's iterations while any lane of the wave
// needs them, up to newton_max_iter in all.  A lane has converged once one of
// its steps is within newton_tol; later iterations only move it by rounding.
// A singular Jacobian or a non-finite iterate leaves NaNs, which report
// non-convergence.

template <int D>
struct Element;

// In a cell whose element is close to a parallelogram (the common case)
// Newton from the linear root converges in about three iterations.
constexpr int kFastNewton = 3;


__device__ __forceinline__ double rcp_refined(double d) {
  const double r = __builtin_amdgcn_rcp(d);
  return fma(r, fma(-d, r, 1.0), r);
}

template <>
struct Element<2> {
  double v0[2], a[2], b[2], c[2];

  __device__ __forceinline__ void set(const double (*V)[2]) {
    for (int i = 0; i < 2; ++i) {
      v0[i] = V[0][i];
      a[i] = V[1][i] - V[0][i];
      b[i] = V[2][i] - V[0][i];
      c[i] = (V[3][i] - V[1][i]) - (V[2][i] - V[0][i]);
    }
  }

  __device__ __forceinline__ int solve(const GridArgs& g, double* xi) const {
    const double det = a[0] * b[1] - b[0] * a[1];
    if (!(det != 0.0) || !isfinite(det)) return -1;
    const double inv = rcp_refined(det);
    const double xl = (-v0[0] * b[1] + b[0] * v0[1]) * inv;
    const double yl = (-a[0] * v0[1] + v0[0] * a[1]) * inv;
    double x = xl, y = yl;
    bool conv = false;
    // Newton's iteration, then chord iterations with its Jacobian (as in
    // Element<3>::solve).
    double j00 = 0.0, j01 = 0.0, j10 = 0.0, j11 = 0.0, ij = 0.0;
    const auto step = [&]() {
      const double f0 = v0[0] + a[0] * x + b[0] * y + c[0] * (x * y);
      const double f1 = v0[1] + a[1] * x + b[1] * y + c[1] * (x * y);
      const double dx = (f0 * j11 - j01 * f1) * ij;
      const double dy = (j00 * f1 - f0 * j10) * ij;
      x -= dx;
      y -= dy;
      conv = conv || fmax(fabs(dx), fabs(dy)) <= g.newton_tol;
    };
    const auto newton = [&]() {
      j00 = a[0] + c[0] * y;
      j01 = b[0] + c[0] * x;
      j10 = a[1] + c[1] * y;
      j11 = b[1] + c[1] * x;
      ij = rcp_refined(j00 * j11 - j01 * j10);
      step();
    };
    if (g.newton_max_iter > 0) newton();
#pragma unroll
    for (int it = 1; it < kFastNewton; ++it)
      if (it < g.newton_max_iter) step();
    for (int it = kFastNewton; it < g.newton_max_iter && __ballot(!conv) != 0ull; ++it)
      newton();
    if (conv && isfinite(x) && isfinite(y)) {
      xi[0] = x;
      xi[1] = y;
      return 1;
    }
    xi[0] = xl;
    xi[1] = yl;
    return 0;
  }
};

template <>
struct Element<3> {
  double v0[3], a[3], b[3], c[3], ab[3], ac[3], bc[3], abc[3];

  __device__ __forceinline__ void set(const double (*V)[3]) {
    for (int i = 0; i < 3; ++i) {
      v0[i] = V[0][i];
      a[i] = V[1][i] - V[0][i];
      b[i] = V[2][i] - V[0][i];
      c[i] = V[4][i] - V[0][i];
      ab[i] = (V[3][i] - V[1][i]) - (V[2][i] - V[0][i]);
      ac[i] = (V[5][i] - V[1][i]) - (V[4][i] - V[0][i]);
      bc[i] = (V[6][i] - V[2][i]) - (V[4][i] - V[0][i]);
      abc[i] = ((V[7][i] - V[6][i]) - (V[5][i] - V[4][i])) -
               ((V[3][i] - V[2][i]) - (V[1][i] - V[0][i]));
    }
  }

  __device__ __forceinline__ static void cross(const double* p, const double* q, double* o) {
    o[0] = p[1] * q[2] - p[2] * q[1];
    o[1] = p[2] * q[0] - p[0] * q[2];
    o[2] = p[0] * q[1] - p[1] * q[0];
  }

  __device__ __forceinline__ static double dot(const double* p, const double* q) {
    return p[0] * q[0] + p[1] * q[1] + p[2] * q[2];
  }

  // Linear systems by Cramer's rule: M d = f for M with columns (c0, c1, c2)
  // is d_k = f . (c_{k+1} x c_{k+2}) / det.
  __device__ __forceinline__ int solve(const GridArgs& g, double* xi) const {
    double x12[3], x20[3], x01[3];
    cross(b, c, x12);
    cross(c, a, x20);
    cross(a, b, x01);
    const double det = dot(a, x12);
    if (!(det != 0.0) || !isfinite(det)) return -1;
    const double inv = rcp_refined(det);
    const double xl = -dot(v0, x12) * inv, yl = -dot(v0, x20) * inv, zl = -dot(v0, x01) * inv;
    double x = xl, y = yl, z = zl;
    bool conv = false;
    // Newton's iteration; `keep` stores its Jacobian's cofactors and
    // reciprocal determinant for the chord iterations.
    double k12[3], k20[3], k01[3], ij = 0.0;
    const auto residual = [&](double* f) {
#pragma unroll
      for (int i = 0; i < 3; ++i)
        f[i] = v0[i] + a[i] * x + b[i] * y + c[i] * z + ab[i] * (x * y) + ac[i] * (x * z) +
               bc[i] * (y * z) + abc[i] * (x * y * z);
    };
    const auto step = [&](const double* f) {
      const double dx = dot(f, k12) * ij, dy = dot(f, k20) * ij, dz = dot(f, k01) * ij;
      x -= dx;
      y -= dy;
      z -= dz;
      conv = conv || fmax(fabs(dx), fmax(fabs(dy), fabs(dz))) <= g.newton_tol;
    };
    const auto newton = [&]() {
      double f[3], j0[3], j1[3], j2[3];
      residual(f);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        j0[i] = a[i] + ab[i] * y + ac[i] * z + abc[i] * (y * z);
        j1[i] = b[i] + ab[i] * x + bc[i] * z + abc[i] * (x * z);
        j2[i] = c[i] + ac[i] * x + bc[i] * y + abc[i] * (x * y);
      }
      cross(j1, j2, k12);
      cross(j2, j0, k20);
      cross(j0, j1, k01);
      ij = rcp_refined(dot(j0, k12));
      step(f);
    };
    // The first kFastNewton iterations run unconditionally: Newton's, then
    // chord iterations with its Jacobian, which from the linear root cut the
    // error by about the element's non-affine part times the first step
    // each.  Lanes not converged after them continue with Newton's
    // iterations while any lane of the wave needs them.
    if (g.newton_max_iter > 0) newton();
#pragma unroll
    for (int it = 1; it < kFastNewton; ++it)
      if (it < g.newton_max_iter) {
        double f[3];
        residual(f);
        step(f);
      }
    for (int it = kFastNewton; it < g.newton_max_iter && __ballot(!conv) != 0ull; ++it)
      newton();
    if (conv && isfinite(x) && isfinite(y) && isfinite(z)) {
      xi[0] = x;
      xi[1] = y;
      xi[2] = z;
      return 1;
    }
    xi[0] = xl;
    xi[1] = yl;
    xi[2] = zl;
    return 0;
  }
};

// Result codes of locate().
enum { LOC_OK = 0, LOC_SEARCH_FAIL = 1, LOC_NEWTON_FAIL = 2 };

template <int D>
__device__ __forceinline__ bool in_cube(const GridArgs& g, const double* xi) {
  bool ok = true;
#pragma unroll
  for (int a = 0; a < D; ++a) ok = ok && (xi[a] >= -g.eps) && (xi[a] <= 1.0 + g.eps);
  return ok;
}

// Element with lower vertex r for target mesh node tgt; `disp(v, d)` returns
// the displacement (cells) of the lattice node with unwrapped index v.
// Returns Element::solve's code.
template <int D, class DispFn>
__device__ __forceinline__ int element_solve(const GridArgs& g, const DispFn& disp,
                                             const int* tgt, const int* r, double* xi) {
  double V[1 << D][D];
#pragma unroll
  for (int e = 0; e < (1 << D); ++e) {
    int v[D];
#pragma unroll
    for (int a = 0; a < D; ++a) v[a] = r[a] + ((e >> a) & 1);
    double d[D];
    disp(v, d);
#pragma unroll
    for (int a = 0; a < D; ++a) V[e][a] = (double)(v[a] - tgt[a]) + d[a];
  }
  Element<D> el;
  el.set(V);
  return el.solve(g, xi);
}

// Host-element search (Sec. 2.2) after the first attempt: rc0 / x0 are the
// solve result in the start cell r (the cell below tgt - d(tgt)).  The search
// moves one cell per axis toward the side an out-of-range local coordinate
// points to.  A cell is accepted only when Newton converges inside its unit
// cube; when Newton does not converge the linear root points the way.  If
// the walk stalls (linear root inside, Newton not converging) or does not
// settle within walk_max moves, the cells of the box of half-width
// scan_radius around the start cell are tried in order, x fastest.
// `solve(r, x)` solves in cell r (Element::solve's code).  On return r is the
// host cell; `walked` reports 0 (start cell), 1 (walked), 2 (fallback scan).
template <int D, class SolveFn>
__device__ __forceinline__ int locate_from(const GridArgs& g, const SolveFn& solve, int rc0,
                                           const double* x0, int* r, double* xi, int& walked) {
  int start[D];
  double x[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    start[a] = r[a];
    x[a] = x0[a];
  }
  walked = 0;
  bool newton_trouble = false;
  int rc = rc0;
  for (int walk = 0; walk < g.walk_max; ++walk) {
    if (walk > 0) rc = solve(r, x);
    if (rc < 0) break;
    if (in_cube<D>(g, x)) {
      if (rc == 1) {
#pragma unroll
        for (int a = 0; a < D; ++a) xi[a] = x[a];
        return LOC_OK;
      }
      newton_trouble = true;
      break;
    }
#pragma unroll
    for (int a = 0; a < D; ++a) r[a] += (x[a] < -g.eps) ? -1 : ((x[a] > 1.0 + g.eps) ? 1 : 0);
    walked = 1;
  }
  const int W = g.scan_radius, span = 2 * g.scan_radius + 1;
  int cnt = 1;
  for (int a = 0; a < D; ++a) cnt *= span;
  for (int q = 0; q < cnt; ++q) {
    int qq = q;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      r[a] = start[a] - W + qq % span;
      qq /= span;
    }
    rc = solve(r, x);
    if (rc >= 0 && in_cube<D>(g, x)) {
      if (rc == 1) {
#pragma unroll
        for (int a = 0; a < D; ++a) xi[a] = x[a];
        walked = 2;
        return LOC_OK;
      }
      newton_trouble = true;
    }
  }
  return newton_trouble ? LOC_NEWTON_FAIL : LOC_SEARCH_FAIL;
}

// Jump criterion of Sec. 2.3 on one axis, evaluated in FP64 from the stored
// values: |h+ - 2h + h-| > theta * max(|h+ - h|, |h - h-|).
__device__ __forceinline__ bool jump_flag(double hm, double hc, double hp, double theta) {
#pragma clang fp contract(off)
  const double d2 = (hp - 2.0 * hc) + hm;
  const double dp = hp - hc;
  const double dm = hc - hm;
  return fabs(d2) > theta * fmax(fabs(dp), fabs(dm));
}

}  // namespace sl
