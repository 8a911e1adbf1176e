// Trajectory integration of the material lattice (Sec. 2, eqs. "momento" and
// "vel"): one work-item per lattice node, fourth-order Runge-Kutta or the
// low-storage third-order scheme of Williamson, FP64 displacement in cell
// units, structure-of-arrays.
#pragma once

#include "sl_device.h"

namespace sl {

constexpr int kBlock = 256;

template <int D>
__device__ __forceinline__ void unflatten(const GridArgs& g, int lin, int* idx) {
  idx[0] = lin % g.n[0];
  if constexpr (D == 2) {
    idx[1] = lin / g.n[0];
  } else {
    const int q = lin / g.n[0];
    idx[1] = q % g.n[1];
    idx[2] = q / g.n[1];
  }
}

template <int D>
__device__ __forceinline__ int flatten(const GridArgs& g, const int* w) {
  if constexpr (D == 2)
    return w[0] + g.n[0] * w[1];
  else
    return w[0] + g.n[0] * (w[1] + g.n[1] * w[2]);
}

// ---------------------------------------------------------------------------
// Trajectories (Sec. 2, eq. "vel").

// Time factors cos(pi t_s / p0) of the periodic families at the stage times,
// computed on the host (1 for the steady families).
struct StageTimes {
  double tf[4];
};

// Launched on a (ceil(nx/64), ceil(ny/4), nz) grid of 64 x 4 work-items, so
// node coordinates come without integer division.
constexpr int kTrajBX = 64, kTrajBY = 4;

// Trajectory of lattice node idx over one step (or one more step when
// `accumulate` is set), with the velocity evaluator `vel` (init(x0), then
// eval(v, x0, delta, tf, u) at x0 + delta).
// `trig` (fresh lattice only): the per-axis sin/cos table of trig_table_kernel
// for the velocity families whose evaluator starts from sin/cos at x0.
// traj_start reads the start position and initialises `vel`; traj_finish
// integrates from there and writes the displacement.  Split so that a caller
// can issue the evaluator's table loads first, then loads of its own, and
// integrate while those are in flight.
template <int D, class Vel>
__device__ __forceinline__ void traj_start(const GridArgs& g, const VelArgs& v, Vel& vel,
                                           const double* __restrict__ disp, double dt,
                                           int accumulate, const int* idx,
                                           const double* __restrict__ trig, double* d,
                                           double* x) {
  const int lin = flatten<D>(g, idx);
#pragma unroll
  for (int a = 0; a < D; ++a) {
    d[a] = accumulate ? disp[(size_t)a * g.ntot + lin] : 0.0;
    x[a] = ((double)(idx[a] + g.off[a]) + d[a]) * g.h[a];
  }
  const bool small = dt * v.shift_rate <= kSmallShift;
  if (trig && !accumulate)
    vel.init_table(trig, g, idx, small);
  else
    vel.init(v, x, small);
}

template <int D, class Vel>
__device__ __forceinline__ void traj_finish(const GridArgs& g, const VelArgs& v, const Vel& vel,
                                            double* __restrict__ disp, const StageTimes& st,
                                            double dt, int integrator, const int* idx, double* d,
                                            const double* x) {
  const int lin = flatten<D>(g, idx);
  if (integrator == SL_RK4) {
    double k1[D], k2[D], k3[D], k4[D], o[D];
    vel.eval(v, x, nullptr, st.tf[0], k1);
#pragma unroll
    for (int a = 0; a < D; ++a) o[a] = 0.5 * dt * k1[a];
    vel.eval(v, x, o, st.tf[1], k2);
#pragma unroll
    for (int a = 0; a < D; ++a) o[a] = 0.5 * dt * k2[a];
    vel.eval(v, x, o, st.tf[1], k3);
#pragma unroll
    for (int a = 0; a < D; ++a) o[a] = dt * k3[a];
    vel.eval(v, x, o, st.tf[2], k4);
    // One quotient per axis: dt (k1 + 2 k2 + 2 k3 + k4) / (6 h), correctly
    // rounded (div_by); 6 h is exact for power-of-two spacings, so uniform
    // translations by whole cells stay exact.
#pragma unroll
    for (int a = 0; a < D; ++a)
      d[a] += div_by(dt * (k1[a] + 2.0 * k2[a] + 2.0 * k3[a] + k4[a]), 6.0 * g.h[a], g.r6h[a]);
  } else {
    // Williamson (1980) 2N-storage RK3: q = A_s q + dt u(x + dx, t + c_s dt),
    // dx += B_s q with A = (0, -5/9, -153/128), B = (1/3, 15/16, 8/15),
    // c = (0, 1/3, 3/4).
    const double A[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
    const double B[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};
    double q[D], dx[D], u[D];
#pragma unroll
    for (int a = 0; a < D; ++a) q[a] = dx[a] = 0.0;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      vel.eval(v, x, s == 0 ? nullptr : dx, st.tf[s], u);
#pragma unroll
      for (int a = 0; a < D; ++a) {
        q[a] = A[s] * q[a] + dt * u[a];
        dx[a] += B[s] * q[a];
      }
    }
#pragma unroll
    for (int a = 0; a < D; ++a) d[a] += div_by(dx[a], g.h[a], g.rh[a]);
  }
#pragma unroll
  for (int a = 0; a < D; ++a) disp[(size_t)a * g.ntot + lin] = d[a];
}

template <int D, class Vel>
__device__ __forceinline__ void traj_node_with(const GridArgs& g, const VelArgs& v, Vel vel,
                                               double* __restrict__ disp,
                                               const StageTimes& st, double dt,
                                               int accumulate, int integrator,
                                               const int* idx,
                                               const double* __restrict__ trig = nullptr) {
  double d[D], x[D];
  traj_start<D>(g, v, vel, disp, dt, accumulate, idx, trig, d, x);
  traj_finish<D>(g, v, vel, disp, st, dt, integrator, idx, d, x);
}

template <int D, int VK>
__device__ __forceinline__ void traj_node(const GridArgs& g, const VelArgs& v,
                                          double* __restrict__ disp, const StageTimes& st,
                                          double dt, int accumulate, int integrator,
                                          const int* idx, const double* trig = nullptr) {
  traj_node_with<D>(g, v, NodeVelocity<VK, D>{}, disp, st, dt, accumulate, integrator, idx,
                    trig);
}

// Does the grid's velocity evaluator start from sin/cos(pi x0) per axis (so
// that a fresh lattice can read them from trig_table_kernel's table)?  (A
// table of the general Fourier encoding's per-mode phase factors e^{i pi c x0}
// was tried for the 3-D Fourier flow: its 16 x 3 loads per node cost more
// than the cosines they replace, 1.99 -> 2.05 ms per 256^3 launch.)
__host__ __device__ inline bool uses_trig_table(const VelArgs& v, int dim) {
  return (v.kind == SL_VEL_SWIRL2D && dim == 2) || (v.kind == SL_VEL_DEFORM3D && dim == 3) ||
         (v.kind == SL_VEL_FOURIER && v.small_k);
}

// Entries (double pairs) of the table: n_x + n_y (+ n_z).
__host__ __device__ inline size_t trig_table_pairs(const GridArgs& g, int dim) {
  size_t axes = 0;
  for (int a = 0; a < dim; ++a) axes += (size_t)g.n[a];
  return axes;
}

// sin/cos of pi times the first-stage argument of the evaluator, per axis a
// and mesh index i: x0 = (i + off_a) h_a (the Fourier ik encoding takes
// x0 * kscale_a).  Layout: axis a holds sin at [base_a, base_a + n_a) and cos
// at [base_a + n_a, base_a + 2 n_a), base_a = 2 sum_{b<a} n_b.  The values are
// the ones NodeVelocity::init computes for a lattice node on its mesh node,
// by the same expressions.
template <int D>
__global__ __launch_bounds__(kBlock) void trig_table_kernel(GridArgs g, VelArgs v,
                                                            double* __restrict__ trig) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int a = 0, base = 0;
  while (a < D && i >= g.n[a]) {
    i -= g.n[a];
    base += 2 * g.n[a];
    ++a;
  }
  if (a >= D) return;
  const double x0 = ((double)(i + g.off[a]) + 0.0) * g.h[a];
  const double arg = v.kind == SL_VEL_FOURIER ? x0 * v.kscale[a] : x0;
  double s, c;
  sincospi(arg, &s, &c);
  trig[base + i] = s;
  trig[base + g.n[a] + i] = c;
}

// Fills the grid's table (host side; `tab` holds trig_table_pairs pairs).
template <int D>
inline hipError_t launch_trig_table(const GridArgs& g, const VelArgs& v, double* tab,
                                    hipStream_t s) {
  const size_t n = trig_table_pairs(g, D);
  trig_table_kernel<D><<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(g, v, tab);
  return hipGetLastError();
}

// Gridded velocity in 2-D with the samples around a tile staged in LDS: the
// same Z-spline sum as velocity<SL_VEL_GRIDDED> (same weights, same order of
// taps), read from the box [bx0, bx0 + W) x [by0, by0 + W) of mesh nodes
// (unwrapped coordinates) when the point's window lies in it, else from global
// memory.
struct GriddedBox2D {
  const double* box;  // 2 planes of W x W samples
  int bx0, by0, W;

  __device__ __forceinline__ void init(const VelArgs&, const double*, bool) {}
  __device__ __forceinline__ void init_table(const double*, const GridArgs&, const int*, bool) {}

  __device__ __forceinline__ void eval(const VelArgs& v, const double* x0, const double* delta,
                                       double, double* u) const {
    int r[2];
    double w[2][6];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const double xa = delta ? x0[a] + delta[a] : x0[a];
      const double sa = xa / v.ug_h[a];
      r[a] = (int)floor(sa);
      zspline_weights<double>(v.ug_m, sa - (double)r[a], w[a]);
    }
    u[0] = u[1] = 0.0;
    const int lo = 2 - v.ug_m, hi = 3 + v.ug_m;
    const int ox = r[0] - 2 - bx0, oy = r[1] - 2 - by0;  // window origin in the box
    const bool in = ox + lo >= 0 && oy + lo >= 0 && ox + hi < W && oy + hi < W;
    const int nx = v.ug_n[0], ny = v.ug_n[1];
#pragma unroll
    for (int ky = 0; ky < 6; ++ky) {
      if (ky < lo || ky > hi) continue;
      double sx[2] = {0.0, 0.0};
      if (in) {
        const int row = (oy + ky) * W + ox;
#pragma unroll
        for (int kx = 0; kx < 6; ++kx) {
          if (kx < lo || kx > hi) continue;
#pragma unroll
          for (int a = 0; a < 2; ++a) sx[a] = fma(box[a * W * W + row + kx], w[0][kx], sx[a]);
        }
      } else {
        const int grow = nx * wrap_index(r[1] - 2 + ky, ny);
#pragma unroll
        for (int kx = 0; kx < 6; ++kx) {
          if (kx < lo || kx > hi) continue;
          const int lin = grow + wrap_index(r[0] - 2 + kx, nx);
#pragma unroll
          for (int a = 0; a < 2; ++a) sx[a] = fma(v.ug[a][lin], w[0][kx], sx[a]);
        }
      }
      // In 2-D the gridded sum's y-z weight is w_y * 1.
#pragma unroll
      for (int a = 0; a < 2; ++a) u[a] = fma(sx[a], w[1][ky] * 1.0, u[a]);
    }
  }
};

// Tiles of the 2-D gridded trajectory kernel: 16 x 16 lattice nodes and a box
// reaching kGridMargin nodes beyond them on every side (stage points up to
// kGridMargin - 3 cells from their node keep their windows in the box).
constexpr int kGridTile = 16, kGridMargin = 8, kGridBox = kGridTile + 2 * kGridMargin;

template <int D>
__global__ __launch_bounds__(256) void traj_gridded2d_kernel(GridArgs g, VelArgs v,
                                                             double* __restrict__ disp,
                                                             StageTimes st, double dt,
                                                             int accumulate, int integrator,
                                                             int tiles_x) {
  static_assert(D == 2, "2-D grids only");
  __shared__ double sbox[2 * kGridBox * kGridBox];
  const int i0 = (blockIdx.x % tiles_x) * kGridTile, j0 = (blockIdx.x / tiles_x) * kGridTile;
  const int bx0 = i0 - kGridMargin, by0 = j0 - kGridMargin;
  const int nx = g.n[0], ny = g.n[1];
  constexpr int NB = kGridBox * kGridBox;
  for (int e = threadIdx.x; e < NB; e += 256) {
    const int gy = e / kGridBox, gx = e - gy * kGridBox;
    const int lin = wrap_index(by0 + gy, ny) * nx + wrap_index(bx0 + gx, nx);
    sbox[e] = v.ug[0][lin];
    sbox[NB + e] = v.ug[1][lin];
  }
  __syncthreads();
  const int idx[2] = {i0 + (int)(threadIdx.x % kGridTile), j0 + (int)(threadIdx.x / kGridTile)};
  if (idx[0] >= nx || idx[1] >= ny) return;
  traj_node_with<2>(g, v, GriddedBox2D{sbox, bx0, by0, kGridBox}, disp, st, dt, accumulate,
                    integrator, idx);
}


// Trajectory of lattice node idx from its mesh node (a fresh lattice) for
// the grid's velocity family, chosen at run time (a wave-uniform switch).
// Gridded velocities are not integrated here (their interpolation would
// raise the register budget of every kernel that embeds this switch).
template <int D>
__device__ __forceinline__ void traj_any(const GridArgs& g, const VelArgs& v,
                                         double* __restrict__ disp, const StageTimes& st,
                                         double dt, int integrator, const int* idx,
                                         const double* trig = nullptr) {
  switch (v.kind) {
    case SL_VEL_UNIFORM:
      traj_node<D, SL_VEL_UNIFORM>(g, v, disp, st, dt, 0, integrator, idx);
      break;
    case SL_VEL_SOLID_BODY:
      traj_node<D, SL_VEL_SOLID_BODY>(g, v, disp, st, dt, 0, integrator, idx);
      break;
    case SL_VEL_SWIRL2D:
      traj_node<D, SL_VEL_SWIRL2D>(g, v, disp, st, dt, 0, integrator, idx, trig);
      break;
    case SL_VEL_DEFORM3D:
      traj_node<D, SL_VEL_DEFORM3D>(g, v, disp, st, dt, 0, integrator, idx, trig);
      break;
    default:
      traj_node<D, SL_VEL_FOURIER>(g, v, disp, st, dt, 0, integrator, idx,
                                   v.small_k ? trig : nullptr);
      break;
  }
}

// The next step's trajectories, computed by a reconstruction kernel for its
// own tile's lattice nodes: they start on the mesh (the lattice is reset each
// step) and so do not depend on the fields being reconstructed.  `disp` null:
// nothing to do.
// carried: the velocity is transported with the fields (fields 0..dim-1),
// so the next step's displacement of a node is dt times the velocity the
// reconstruction has just produced there, in cells.
struct NextTraj {
  double* disp;
  StageTimes st;
  double dt;
  int integrator;
  int carried;
  const double* trig;  // trig_table_kernel's table, or null
};

// Stand-in for the velocity argument of kernels that never integrate.
struct NoVel {};

// Carried velocity (fields 0..D-1 hold it; no right-hand side): each lattice
// node moves on a straight line with its own velocity, for every integrator.
// Same (64 x 4) grid as traj_kernel.
template <int D, typename T>
__global__ __launch_bounds__(kBlock) void carried_traj_kernel(GridArgs g, FieldPtrs fp,
                                                              double* __restrict__ disp,
                                                              double dt, int accumulate) {
  int idx[D];
  idx[0] = blockIdx.x * kTrajBX + threadIdx.x;
  idx[1] = blockIdx.y * kTrajBY + threadIdx.y;
  if constexpr (D == 3) idx[2] = blockIdx.z;
  if (idx[0] >= g.n[0] || idx[1] >= g.n[1]) return;
  const int lin = flatten<D>(g, idx);
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const double u = (double)static_cast<const T*>(fp.in[a])[lin];
    const double d0 = accumulate ? disp[(size_t)a * g.ntot + lin] : 0.0;
    disp[(size_t)a * g.ntot + lin] = d0 + dt * u / g.h[a];
  }
}

// `trig`: trig_table_kernel's table for a fresh lattice, or null.
template <int D, int VK>
__global__ __launch_bounds__(kBlock) void traj_kernel(GridArgs g, VelArgs v,
                                                      double* __restrict__ disp, StageTimes st,
                                                      double dt, int accumulate,
                                                      int integrator,
                                                      const double* __restrict__ trig) {
  int idx[D];
  idx[0] = blockIdx.x * kTrajBX + threadIdx.x;
  idx[1] = blockIdx.y * kTrajBY + threadIdx.y;
  if constexpr (D == 3) idx[2] = blockIdx.z;
  if (idx[0] >= g.n[0] || idx[1] >= g.n[1]) return;
  traj_node<D, VK>(g, v, disp, st, dt, accumulate, integrator, idx, trig);
}


}  // namespace sl
