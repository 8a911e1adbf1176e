// Source terms (Sec. 2: the right-hand side S_i of eq. "momento" may hold
// spatial derivatives, taken by finite differences on the reference mesh), for
// the 2-D shallow-water system of eq. "nlsw".  A step integrates every lattice
// node's position and values with Williamson's low-storage RK3; each stage
//   1. has the stage fields on the mesh (the fields at t, or the reconstruction
//      of the lattice's stage values),
//   2. evaluates the right-hand side there,
//   3. advances each lattice node with its own velocity and the right-hand
//      side interpolated at its position;
// steps 2 and 3 are one kernel (sw_stage_kernel) that evaluates the
// right-hand side in LDS on the box of mesh nodes its tile's windows cover.
// The host loop in sl.hip runs the reconstructions between the stages and the
// final one that resets the lattice.
#pragma once

#include <limits.h>

#include "sl_device.h"
#include "sl_recon2d.h"

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
  int last;   // last stage: the registers are not needed afterwards
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

// Right-hand side at one mesh node from an accessor G(c, dx, dy) giving
// field c (0: u = u1, 1: v = u2, 2: h) at offset (dx, dy) from the node, and
// the node's y coordinate:
//   S_h = -(1 + h) div u
//   S_u = -h_x + f v + nu V1,   S_v = -h_y - f u + nu V2,
//   V = div[(1 + h)(grad u + grad u^T)]
//     = (1 + h)(lap u + grad div u) + (grad u + grad u^T) grad h.
// Pure second derivatives use the second-derivative rule, mixed ones the
// product of the first-derivative rules.  Every caller goes through this
// function, so the result at a node does not depend on where G comes from.
template <int M, typename Acc>
__device__ __forceinline__ void sw_rhs(const SrcArgs& a, double ihx, double ihy, double y,
                                       const Acc& G, double* out) {
  constexpr int W = 2 * M + 1;
  double ux = 0.0, uy = 0.0, vx = 0.0, vy = 0.0, hx = 0.0, hy = 0.0;
#pragma unroll
  for (int k = 0; k < W; ++k) {
    if (k == M) continue;
    const double c = fd_d1<M>(k);
    ux = fma(c, G(0, k - M, 0), ux);
    vx = fma(c, G(1, k - M, 0), vx);
    hx = fma(c, G(2, k - M, 0), hx);
    uy = fma(c, G(0, 0, k - M), uy);
    vy = fma(c, G(1, 0, k - M), vy);
    hy = fma(c, G(2, 0, k - M), hy);
  }
  ux *= ihx;
  vx *= ihx;
  hx *= ihx;
  uy *= ihy;
  vy *= ihy;
  hy *= ihy;
  const double u = G(0, 0, 0), v = G(1, 0, 0), h = G(2, 0, 0);
  const double f = a.fc + a.beta * (y - a.y0);
  double s_u = -hx + f * v;
  double s_v = -hy - f * u;
  const double s_h = -(1.0 + h) * (ux + vy);
  if (a.nu != 0.0) {
    double uxx = 0.0, uyy = 0.0, vxx = 0.0, vyy = 0.0, uxy = 0.0, vxy = 0.0;
#pragma unroll
    for (int k = 0; k < W; ++k) {
      const double c = fd_d2<M>(k);
      uxx = fma(c, G(0, k - M, 0), uxx);
      vxx = fma(c, G(1, k - M, 0), vxx);
      uyy = fma(c, G(0, 0, k - M), uyy);
      vyy = fma(c, G(1, 0, k - M), vyy);
    }
#pragma unroll
    for (int l = 0; l < W; ++l) {
      if (l == M) continue;
#pragma unroll
      for (int k = 0; k < W; ++k) {
        if (k == M) continue;
        const double c = fd_d1<M>(k) * fd_d1<M>(l);
        uxy = fma(c, G(0, k - M, l - M), uxy);
        vxy = fma(c, G(1, k - M, l - M), vxy);
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
  out[0] = s_u;
  out[1] = s_v;
  out[2] = s_h;
}

// Stage fields straight from global memory around mesh node (i, j), periodic.
template <typename T>
struct GlobalStage {
  const T* __restrict__ f[3];
  int i, j, nx, ny;
  __device__ __forceinline__ double operator()(int c, int dx, int dy) const {
    return (double)f[c][wrap_index(j + dy, ny) * nx + wrap_index(i + dx, nx)];
  }
};

// Stage fields from the LDS box (FP64, pitch P) at box position (x, y).
struct BoxStage {
  const double* s;
  int plane, P, x, y;
  __device__ __forceinline__ double operator()(int c, int dx, int dy) const {
    return s[c * plane + (y + dy) * P + (x + dx)];
  }
};

// Tiles of the fused stage kernel: 16 x 16 lattice nodes per workgroup.  The
// right-hand side is evaluated on the box of mesh nodes their Z-spline windows
// cover (at most SMAX per side) and the stage fields on that box grown by the
// rule's half-width M; boxes beyond SMAX take the global path.
struct StageTile {
  static constexpr int T = 16;
  static constexpr int SMAX = 24;
};

// One Runge-Kutta stage of every lattice node, fused with the right-hand side:
// the node's velocity is its own stage value (fields 0, 1 of the lattice
// values `fp.out`), the source its stage right-hand side, evaluated on the
// mesh from the stage fields `stage` (fp.in in stage 0) and interpolated at
// the node's stage position with the order-m Z-spline (eq. "multiZ",
// periodic).  Stage 0 starts from the mesh values `fp.in` (every field;
// fields past 2 are passive and only copied) at zero displacement, where the
// interpolation is the node's own value.  Positions and registers are FP64;
// lattice values in T.
template <typename T, int M>
__global__ __launch_bounds__(256) void sw_stage_kernel(GridArgs g, SrcArgs a, SrcStage st,
                                                       FieldPtrs fp, const T* __restrict__ s0,
                                                       const T* __restrict__ s1,
                                                       const T* __restrict__ s2,
                                                       double* __restrict__ disp,
                                                       double* __restrict__ qx,
                                                       double* __restrict__ qh, int tiles_x,
                                                       int ntiles) {
  constexpr int TT = StageTile::T, SMAX = StageTile::SMAX, GMAX = SMAX + 2 * M;
  __shared__ double sG[3 * GMAX * GMAX];
  __shared__ double sS[3 * SMAX * SMAX];
  __shared__ int box[4];
  const int nx = g.n[0], ny = g.n[1];
  const size_t N = (size_t)g.ntot;
  const int tile = xcd_tile(blockIdx.x, ntiles);
  const int i0 = (tile % tiles_x) * TT, j0 = (tile / tiles_x) * TT;
  const int tx = threadIdx.x % TT, ty = threadIdx.x / TT;
  const int i = i0 + tx, j = j0 + ty;
  const bool act = i < nx && j < ny;
  const int lin = j * nx + i;
  const double ihx = 1.0 / g.h[0], ihy = 1.0 / g.h[1];

  double d[2] = {0.0, 0.0}, q[2] = {0.0, 0.0}, r[3] = {0.0, 0.0, 0.0}, H[3] = {0.0, 0.0, 0.0};
  if (act) {
    if (st.first) {
#pragma unroll
      for (int f = 0; f < SL_MAX_FIELDS; ++f) {
        if (f >= g.nfields) break;
        const T val = static_cast<const T*>(fp.in[f])[lin];
        if (f < 3) H[f] = (double)val;
        else static_cast<T*>(fp.out[f])[lin] = val;
      }
    } else {
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        d[c] = disp[c * N + lin];
        q[c] = qx[c * N + lin];
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        r[c] = qh[c * N + lin];
        H[c] = (double)static_cast<const T*>(fp.out[c])[lin];
      }
    }
  }
  // Window base of each node (slot k of the six holds node base - 2 + k) and
  // the box of mesh nodes the tile's windows cover.  In stage 0 the weights
  // select the node itself, so the box is the tile.
  int base[2];
  double w[2][6];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const double p = (double)(c == 0 ? i : j) + d[c];
    const double fl = floor(p);
    base[c] = (int)fl;
    zspline_weights<double>(g.order_max, p - fl, w[c]);
  }
  if (threadIdx.x == 0) {
    box[0] = box[1] = INT_MAX;
    box[2] = box[3] = INT_MIN;
  }
  __syncthreads();
  const int lo = st.first ? 0 : -2, hi = st.first ? 0 : 3;
  {
    const int bx0 = wave_min(act ? base[0] + lo : INT_MAX);
    const int by0 = wave_min(act ? base[1] + lo : INT_MAX);
    const int bx1 = wave_max(act ? base[0] + hi : INT_MIN);
    const int by1 = wave_max(act ? base[1] + hi : INT_MIN);
    if ((threadIdx.x & 63) == 0) {
      atomicMin(&box[0], bx0);
      atomicMin(&box[1], by0);
      atomicMax(&box[2], bx1);
      atomicMax(&box[3], by1);
    }
  }
  __syncthreads();
  const int bx0 = box[0], by0 = box[1];
  const int SBX = box[2] - bx0 + 1, SBY = box[3] - by0 + 1;
  const T* stg[3] = {s0, s1, s2};
  double s_hat[3] = {0.0, 0.0, 0.0};
  if (SBX <= SMAX && SBY <= SMAX) {
    // Stage fields of the box grown by M into LDS (FP64), wrapped.
    const int GBX = SBX + 2 * M, GBY = SBY + 2 * M, gplane = GBX * GBY;
    for (int e = threadIdx.x; e < gplane; e += blockDim.x) {
      const int gy = e / GBX, gx = e - gy * GBX;
      const int at = wrap_index(by0 - M + gy, ny) * nx + wrap_index(bx0 - M + gx, nx);
#pragma unroll
      for (int c = 0; c < 3; ++c) sG[c * gplane + e] = (double)stg[c][at];
    }
    __syncthreads();
    // Right-hand side on the box.
    const int splane = SBX * SBY;
    for (int e = threadIdx.x; e < splane; e += blockDim.x) {
      const int sy = e / SBX, sx = e - sy * SBX;
      const BoxStage acc{sG, gplane, GBX, sx + M, sy + M};
      double o[3];
      sw_rhs<M>(a, ihx, ihy, (double)wrap_index(by0 + sy, ny) * g.h[1], acc, o);
#pragma unroll
      for (int c = 0; c < 3; ++c) sS[c * splane + e] = o[c];
    }
    __syncthreads();
    if (act) {
      if (st.first) {
        const int e = (j - by0) * SBX + (i - bx0);
#pragma unroll
        for (int c = 0; c < 3; ++c) s_hat[c] = sS[c * splane + e];
      } else {
        const int ow = 2 - g.order_max, hw = 3 + g.order_max;
#pragma unroll
        for (int ky = 0; ky < 6; ++ky) {
          if (ky < ow || ky > hw) continue;
          const int row = (base[1] - 2 + ky - by0) * SBX + (base[0] - 2 - bx0);
          double sx[3] = {0.0, 0.0, 0.0};
#pragma unroll
          for (int kx = 0; kx < 6; ++kx) {
            if (kx < ow || kx > hw) continue;
#pragma unroll
            for (int c = 0; c < 3; ++c) sx[c] = fma(sS[c * splane + row + kx], w[0][kx], sx[c]);
          }
#pragma unroll
          for (int c = 0; c < 3; ++c) s_hat[c] = fma(sx[c], w[1][ky], s_hat[c]);
        }
      }
    }
  } else if (act) {
    // Box too large for LDS: the right-hand side of each tap from global
    // memory (the same arithmetic).
    const int ow = st.first ? 2 : 2 - g.order_max, hw = st.first ? 2 : 3 + g.order_max;
#pragma unroll 1
    for (int ky = 0; ky < 6; ++ky) {
      if (ky < ow || ky > hw) continue;
      const int yy = wrap_index(base[1] - 2 + ky, ny);
      double sx[3] = {0.0, 0.0, 0.0};
#pragma unroll 1
      for (int kx = 0; kx < 6; ++kx) {
        if (kx < ow || kx > hw) continue;
        const int xx = wrap_index(base[0] - 2 + kx, nx);
        const GlobalStage<T> acc{{s0, s1, s2}, xx, yy, nx, ny};
        double o[3];
        sw_rhs<M>(a, ihx, ihy, (double)yy * g.h[1], acc, o);
        double wx = w[0][5];
#pragma unroll
        for (int k = 4; k >= 0; --k) wx = kx == k ? w[0][k] : wx;
#pragma unroll
        for (int c = 0; c < 3; ++c) sx[c] = fma(o[c], wx, sx[c]);
      }
      double wy = w[1][5];
#pragma unroll
      for (int k = 4; k >= 0; --k) wy = ky == k ? w[1][k] : wy;
#pragma unroll
      for (int c = 0; c < 3; ++c) s_hat[c] = fma(sx[c], wy, s_hat[c]);
    }
  }
  if (!act) return;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    q[c] = st.A * q[c] + st.dt * H[c] / g.h[c];
    d[c] += st.B * q[c];
    disp[c * N + lin] = d[c];
    if (!st.last) qx[c * N + lin] = q[c];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    r[c] = st.A * r[c] + st.dt * s_hat[c];
    if (!st.last) qh[c * N + lin] = r[c];
    static_cast<T*>(fp.out[c])[lin] = (T)(H[c] + st.B * r[c]);
  }
}

}  // namespace sl
