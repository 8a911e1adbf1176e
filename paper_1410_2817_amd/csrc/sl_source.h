// Source terms (Sec. 2: the right-hand side S_i of eq. "momento" may hold
// spatial derivatives, taken by finite differences on the reference mesh), for
// the 2-D shallow-water system of eq. "nlsw".  A step integrates every lattice
// node's position and values with Williamson's low-storage RK3; each stage
//   1. has the stage fields on the mesh (the fields at t, or the reconstruction
//      of the lattice's stage values),
//   2. evaluates the right-hand side there (sw_source_kernel),
//   3. advances each lattice node with its own velocity and the right-hand
//      side interpolated at its position (sw_stage_kernel).
// The host loop in sl.hip runs the reconstructions between the stages and the
// final one that resets the lattice.
#pragma once

#include "sl_device.h"
#include "sl_traj.h"

namespace sl {

// f = fc + beta (y - y0): the paper's equatorial beta plane is fc = 0,
// beta = f0, y0 the equator; nu the viscosity.
struct SrcArgs {
  double fc, beta, y0, nu;
};

// One Runge-Kutta stage: q = A q + dt F, y += B q (A = 0 in stage 0).
struct SrcStage {
  double A, B, dt;
  int first;  // stage 0: start from the mesh values, zero registers
};

// Centred (2M+1)-point rules on a unit grid, offset k - M: first derivative
// (1/2 (-1, 0, 1); 1/12 (1, -8, 0, 8, -1)) and second derivative ((1, -2, 1);
// 1/12 (-1, 16, -30, 16, -1)).  Constant-folded after unrolling.
template <int M>
__device__ __forceinline__ constexpr double fd_d1(int k) {
  if constexpr (M == 1) {
    return k == 0 ? -0.5 : (k == 2 ? 0.5 : 0.0);
  } else {
    return k == 0 ? 1.0 / 12 : k == 1 ? -8.0 / 12 : k == 3 ? 8.0 / 12 : k == 4 ? -1.0 / 12 : 0.0;
  }
}
template <int M>
__device__ __forceinline__ constexpr double fd_d2(int k) {
  if constexpr (M == 1) {
    return k == 1 ? -2.0 : 1.0;
  } else {
    return k == 0 || k == 4 ? -1.0 / 12 : k == 1 || k == 3 ? 16.0 / 12 : -30.0 / 12;
  }
}

// Right-hand side on the mesh, one work-item per node: u = G0, v = G1 (the
// carried velocity), h = G2.
//   S_h = -(1 + h) div u
//   S_u = -h_x + f v + nu V1,   S_v = -h_y - f u + nu V2,
//   V = div[(1 + h)(grad u + grad u^T)]
//     = (1 + h)(lap u + grad div u) + (grad u + grad u^T) grad h.
// Pure second derivatives use the second-derivative rule, mixed ones the
// product of the first-derivative rules.
template <typename T, int M>
__global__ __launch_bounds__(kBlock) void sw_source_kernel(GridArgs g, SrcArgs a,
                                                           const T* __restrict__ gu,
                                                           const T* __restrict__ gv,
                                                           const T* __restrict__ gh,
                                                           double* __restrict__ su,
                                                           double* __restrict__ sv,
                                                           double* __restrict__ sh) {
  const int i = blockIdx.x * kTrajBX + threadIdx.x;
  const int j = blockIdx.y * kTrajBY + threadIdx.y;
  if (i >= g.n[0] || j >= g.n[1]) return;
  const int nx = g.n[0], ny = g.n[1];
  constexpr int W = 2 * M + 1;
  int xo[W], yo[W];
#pragma unroll
  for (int k = 0; k < W; ++k) {
    xo[k] = wrap_index(i + k - M, nx);
    yo[k] = wrap_index(j + k - M, ny) * nx;
  }
  const int row = j * nx, lin = row + i;
  const double ihx = 1.0 / g.h[0], ihy = 1.0 / g.h[1];
  double ux = 0.0, uy = 0.0, vx = 0.0, vy = 0.0, hx = 0.0, hy = 0.0;
#pragma unroll
  for (int k = 0; k < W; ++k) {
    if (k == M) continue;
    const double c = fd_d1<M>(k);
    ux = fma(c, (double)gu[row + xo[k]], ux);
    vx = fma(c, (double)gv[row + xo[k]], vx);
    hx = fma(c, (double)gh[row + xo[k]], hx);
    uy = fma(c, (double)gu[yo[k] + i], uy);
    vy = fma(c, (double)gv[yo[k] + i], vy);
    hy = fma(c, (double)gh[yo[k] + i], hy);
  }
  ux *= ihx;
  vx *= ihx;
  hx *= ihx;
  uy *= ihy;
  vy *= ihy;
  hy *= ihy;
  const double u = (double)gu[lin], v = (double)gv[lin], h = (double)gh[lin];
  const double f = a.fc + a.beta * ((double)j * g.h[1] - a.y0);
  double s_u = -hx + f * v;
  double s_v = -hy - f * u;
  const double s_h = -(1.0 + h) * (ux + vy);
  if (a.nu != 0.0) {
    double uxx = 0.0, uyy = 0.0, vxx = 0.0, vyy = 0.0, uxy = 0.0, vxy = 0.0;
#pragma unroll
    for (int k = 0; k < W; ++k) {
      const double c = fd_d2<M>(k);
      uxx = fma(c, (double)gu[row + xo[k]], uxx);
      vxx = fma(c, (double)gv[row + xo[k]], vxx);
      uyy = fma(c, (double)gu[yo[k] + i], uyy);
      vyy = fma(c, (double)gv[yo[k] + i], vyy);
    }
#pragma unroll
    for (int l = 0; l < W; ++l) {
      if (l == M) continue;
#pragma unroll
      for (int k = 0; k < W; ++k) {
        if (k == M) continue;
        const double c = fd_d1<M>(k) * fd_d1<M>(l);
        uxy = fma(c, (double)gu[yo[l] + xo[k]], uxy);
        vxy = fma(c, (double)gv[yo[l] + xo[k]], vxy);
      }
    }
    uxx *= ihx * ihx;
    vxx *= ihx * ihx;
    uyy *= ihy * ihy;
    vyy *= ihy * ihy;
    uxy *= ihx * ihy;
    vxy *= ihx * ihy;
    const double V1 = (1.0 + h) * (2.0 * uxx + uyy + vxy) + hx * (2.0 * ux) + hy * (uy + vx);
    const double V2 = (1.0 + h) * (vxx + 2.0 * vyy + uxy) + hx * (vx + uy) + hy * (2.0 * vy);
    s_u = fma(a.nu, V1, s_u);
    s_v = fma(a.nu, V2, s_v);
  }
  su[lin] = s_u;
  sv[lin] = s_v;
  sh[lin] = s_h;
}

// One Runge-Kutta stage of every lattice node (one work-item each).  The
// node's velocity is its own stage value (fields 0, 1 of the lattice values
// `fp.out`), the source its stage right-hand side interpolated at its stage
// position with the order-m Z-spline (eq. "multiZ", periodic).  Stage 0 starts
// from the mesh values `fp.in` (every field; fields past 2 are passive and
// only copied) at zero displacement, where the interpolation is the node's
// own value.  Positions and registers are FP64; lattice values in T.
template <typename T>
__global__ __launch_bounds__(kBlock) void sw_stage_kernel(GridArgs g, SrcStage st, FieldPtrs fp,
                                                          double* __restrict__ disp,
                                                          double* __restrict__ qx,
                                                          double* __restrict__ qh,
                                                          const double* __restrict__ src) {
  const int i = blockIdx.x * kTrajBX + threadIdx.x;
  const int j = blockIdx.y * kTrajBY + threadIdx.y;
  if (i >= g.n[0] || j >= g.n[1]) return;
  const int nx = g.n[0], ny = g.n[1];
  const size_t N = (size_t)g.ntot;
  const int lin = j * nx + i;
  double d[2], q[2], r[3], H[3], s_hat[3];
  if (st.first) {
#pragma unroll
    for (int f = 0; f < SL_MAX_FIELDS; ++f) {
      if (f >= g.nfields) break;
      const T val = static_cast<const T*>(fp.in[f])[lin];
      if (f < 3) H[f] = (double)val;
      else static_cast<T*>(fp.out[f])[lin] = val;
    }
#pragma unroll
    for (int a = 0; a < 2; ++a) d[a] = q[a] = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      r[c] = 0.0;
      s_hat[c] = src[c * N + lin];
    }
  } else {
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      d[a] = disp[a * N + lin];
      q[a] = qx[a * N + lin];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      r[c] = qh[c * N + lin];
      H[c] = (double)static_cast<const T*>(fp.out[c])[lin];
    }
    // Z-spline interpolation of the three right-hand sides; slot k holds
    // node floor(p) - 2 + k.
    int base[2];
    double w[2][6];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const double p = (double)(a == 0 ? i : j) + d[a];
      const double fl = floor(p);
      base[a] = (int)fl;
      zspline_weights<double>(g.order_max, p - fl, w[a]);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) s_hat[c] = 0.0;
    const int lo = 2 - g.order_max, hi = 3 + g.order_max;
#pragma unroll
    for (int ky = 0; ky < 6; ++ky) {
      if (ky < lo || ky > hi) continue;
      const int rowo = wrap_index(base[1] - 2 + ky, ny) * nx;
      double sx[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int kx = 0; kx < 6; ++kx) {
        if (kx < lo || kx > hi) continue;
        const int at = rowo + wrap_index(base[0] - 2 + kx, nx);
#pragma unroll
        for (int c = 0; c < 3; ++c) sx[c] = fma(src[c * N + at], w[0][kx], sx[c]);
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) s_hat[c] = fma(sx[c], w[1][ky], s_hat[c]);
    }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    q[a] = st.A * q[a] + st.dt * H[a] / g.h[a];
    d[a] += st.B * q[a];
    disp[a * N + lin] = d[a];
    qx[a * N + lin] = q[a];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    r[c] = st.A * r[c] + st.dt * s_hat[c];
    qh[c * N + lin] = r[c];
    static_cast<T*>(fp.out[c])[lin] = (T)(H[c] + st.B * r[c]);
  }
}

}  // namespace sl
