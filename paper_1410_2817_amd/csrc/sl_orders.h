// Limiter order words (Sec. 2.3) for gfx950.
//
// The limiter's order choice for a mesh node depends only on its host cell r:
// the quintic stencil reads the jump flags of the nodes r-2..r+3 per axis and
// the cubic one those of r-1..r+2.  Both ORs are separable, so short passes
// (one per axis) turn the per-node flag bytes (bit f set when the criterion
// fires for field f along any axis) into one 16-bit word per cell: low byte
// the quintic window, high byte the cubic window, bit f for field f.  The
// reconstruction then reads one word per node.
#pragma once

#include "sl_device.h"
#include "sl_traj.h"

namespace sl {

// Jump flags (Sec. 2.3): bit f of flags[node] is set when the criterion fires
// for field f along any axis.

template <int D, typename T>
__global__ __launch_bounds__(kBlock) void flags_kernel(GridArgs g, FieldPtrs fp,
                                                       uint8_t* __restrict__ flags) {
  const int lin = blockIdx.x * kBlock + threadIdx.x;
  if (lin >= g.ntot) return;
  int idx[D];
  unflatten<D>(g, lin, idx);
  int nb[D][2];
  const int stride[3] = {1, g.n[0], g.n[0] * g.n[1]};
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const int up = idx[a] + 1 == g.n[a] ? -(g.n[a] - 1) : 1;
    const int dn = idx[a] == 0 ? (g.n[a] - 1) : -1;
    nb[a][0] = lin + dn * stride[a];
    nb[a][1] = lin + up * stride[a];
  }
  unsigned bits = 0;
  for (int f = 0; f < g.nfields; ++f) {
    const T* __restrict__ h = static_cast<const T*>(fp.in[f]);
    const double hc = (double)h[lin];
    bool fl = false;
#pragma unroll
    for (int a = 0; a < D; ++a)
      fl = fl || jump_flag((double)h[nb[a][0]], hc, (double)h[nb[a][1]], g.theta);
    bits |= (fl ? 1u : 0u) << f;
  }
  flags[lin] = (uint8_t)bits;
}

// Separable window OR of the jump flags along AXIS.  AXIS 0 reads the flag
// bytes and writes both windows; the y and z passes OR the words' low bytes
// over slots -2..3 and their high bytes over slots -1..2.
template <int AXIS>
__global__ __launch_bounds__(256) void window_or_kernel(GridArgs g,
                                                        const uint8_t* __restrict__ flags,
                                                        const uint16_t* __restrict__ win,
                                                        uint16_t* __restrict__ out) {
  const int x = blockIdx.x * 64 + threadIdx.x, y = blockIdx.y * 4 + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= g.n[0] || y >= g.n[1]) return;
  const int idx[3] = {x, y, z};
  const int lin = x + g.n[0] * (y + g.n[1] * z);
  const int n = g.n[AXIS];
  const int stride = AXIS == 0 ? 1 : (AXIS == 1 ? g.n[0] : g.n[0] * g.n[1]);
  const int base = lin - idx[AXIS] * stride;
  int j = idx[AXIS] - 2;
  j = j < 0 ? j + n : j;  // n >= 6
  unsigned lo = 0, hi = 0;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const unsigned v = AXIS == 0 ? (unsigned)flags[base + j] * 0x101u
                                 : (unsigned)win[base + j * stride];
    lo |= v & 0xffu;
    if (k >= 1 && k <= 4) hi |= v & 0xff00u;
    j = j + 1 == n ? 0 : j + 1;
  }
  out[lin] = (uint16_t)(lo | hi);
}

// The same passes four x-nodes per work-item, for rows whose length is a
// multiple of 4 (and 16-byte aligned fields): flag bytes and window words
// move as 32- and 64-bit words.

// Flag bytes of the quad x = 4q .. 4q+3 of row (y, z): byte j, bit f set when
// the criterion fires for field f at node x + j.
template <int D, typename T>
__device__ __forceinline__ unsigned quad_flag_bits(const GridArgs& g, const FieldPtrs& fp, int q,
                                                   int y, int z) {
  using V4 = T __attribute__((ext_vector_type(4)));
  const int n0 = g.n[0], n1 = g.n[1], n2 = g.n[2];
  const int x = 4 * q;
  const int ym = y == 0 ? n1 - 1 : y - 1, yp = y + 1 == n1 ? 0 : y + 1;
  const int zm = z == 0 ? n2 - 1 : z - 1, zp = z + 1 == n2 ? 0 : z + 1;
  const int rw = n0 * (y + n1 * z);
  const int rym = n0 * (ym + n1 * z), ryp = n0 * (yp + n1 * z);
  const int rzm = n0 * (y + n1 * zm), rzp = n0 * (y + n1 * zp);
  const int xm = x == 0 ? n0 - 1 : x - 1, xp = x + 4 == n0 ? 0 : x + 4;
  unsigned bits = 0;
  for (int f = 0; f < g.nfields; ++f) {
    const T* __restrict__ h = static_cast<const T*>(fp.in[f]);
    const V4 c = *reinterpret_cast<const V4*>(h + rw + x);
    const V4 vym = *reinterpret_cast<const V4*>(h + rym + x);
    const V4 vyp = *reinterpret_cast<const V4*>(h + ryp + x);
    const V4 vzm = D == 3 ? *reinterpret_cast<const V4*>(h + rzm + x) : c;
    const V4 vzp = D == 3 ? *reinterpret_cast<const V4*>(h + rzp + x) : c;
    const double l = (double)h[rw + xm], r = (double)h[rw + xp];
    const double cc[4] = {(double)c.x, (double)c.y, (double)c.z, (double)c.w};
    const double am[4] = {(double)vym.x, (double)vym.y, (double)vym.z, (double)vym.w};
    const double ap[4] = {(double)vyp.x, (double)vyp.y, (double)vyp.z, (double)vyp.w};
    const double bm[4] = {(double)vzm.x, (double)vzm.y, (double)vzm.z, (double)vzm.w};
    const double bp[4] = {(double)vzp.x, (double)vzp.y, (double)vzp.z, (double)vzp.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double hm = j == 0 ? l : cc[j - 1], hp = j == 3 ? r : cc[j + 1];
      const bool fl = jump_flag(hm, cc[j], hp, g.theta) ||
                      jump_flag(am[j], cc[j], ap[j], g.theta) ||
                      (D == 3 && jump_flag(bm[j], cc[j], bp[j], g.theta));
      bits |= (fl ? 1u : 0u) << (8 * j + f);
    }
  }
  return bits;
}

// The x window words of a quad from the flag bytes of it and its two
// neighbours (nodes x-4 .. x+7): for node x + j the quintic window ORs bytes
// j+2 .. j+7 (nodes x+j-2 .. x+j+3), the cubic one bytes j+3 .. j+6.
__device__ __forceinline__ unsigned long long quad_window_x(unsigned left, unsigned mid,
                                                            unsigned right) {
  const unsigned w[3] = {left, mid, right};
  unsigned b[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) b[k] = (w[k / 4] >> (8 * (k % 4))) & 0xffu;
  unsigned long long o = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    unsigned lo = 0, hi = 0;
#pragma unroll
    for (int k = 2; k <= 7; ++k) lo |= b[j + k];
#pragma unroll
    for (int k = 3; k <= 6; ++k) hi |= b[j + k];
    o |= (unsigned long long)(lo | (hi << 8)) << (16 * j);
  }
  return o;
}

template <int AXIS>
__global__ __launch_bounds__(256) void window_yz_quad_kernel(
    GridArgs g, const unsigned long long* __restrict__ in4, unsigned long long* __restrict__ out4) {
  const int nq = g.n[0] / 4;
  const int q = blockIdx.x * 64 + threadIdx.x, y = blockIdx.y * 4 + threadIdx.y;
  const int z = blockIdx.z;
  if (q >= nq || y >= g.n[1]) return;
  const int lin = q + nq * (y + g.n[1] * z);
  const int idx = AXIS == 1 ? y : z, n = g.n[AXIS];
  const int stride = AXIS == 1 ? nq : nq * g.n[1];
  const int base = lin - idx * stride;
  int j = idx - 2;
  j = j < 0 ? j + n : j;  // n >= 6
  unsigned long long lo = 0, hi = 0;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const unsigned long long v = in4[base + j * stride];
    lo |= v & 0x00ff00ff00ff00ffull;
    if (k >= 1 && k <= 4) hi |= v & 0xff00ff00ff00ff00ull;
    j = j + 1 == n ? 0 : j + 1;
  }
  out4[lin] = lo | hi;
}

// Flags and x window in one pass (the flag bytes never reach memory), for
// rows of at most kBlock quads: a workgroup holds R = kBlock / nq whole rows
// (nq = n0 / 4 quads per row), so the x neighbours of every quad, the
// periodic ones included, are in its LDS.  Work-item t takes quad t % nq of
// row t / nq.  Grid: (ceil(n1 / R), n2) of kBlock.
template <int D, typename T>
__global__ __launch_bounds__(kBlock) void flags_window_x_kernel(GridArgs g, FieldPtrs fp,
                                                                unsigned long long* __restrict__ out4) {
  __shared__ uint32_t s_f[kBlock];
  const int nq = g.n[0] / 4, R = kBlock / nq;
  const int t = (int)threadIdx.x, q = t % nq, row = t / nq;
  const int y = blockIdx.x * R + row, z = blockIdx.y;
  const bool ok = row < R && y < g.n[1];
  if (ok) s_f[t] = quad_flag_bits<D, T>(g, fp, q, y, z);
  __syncthreads();
  if (!ok) return;
  const int base = row * nq;
  out4[nq * (y + g.n[1] * z) + q] =
      quad_window_x(s_f[base + (q == 0 ? nq - 1 : q - 1)], s_f[t],
                    s_f[base + (q + 1 == nq ? 0 : q + 1)]);
}

// Longer rows: the flag bytes of each quad (grid (ceil(nq/64), ceil(n1/4),
// n2) of 64 x 4), then the x window of each quad from its own and its two
// neighbours' bytes.  (Overlapping segments of 256 quads with the flags in
// LDS, as above, measured slower at 4096^2: 0.645 -> 0.683 ms per step.)
template <int D, typename T>
__global__ __launch_bounds__(256) void flags_quad_kernel(GridArgs g, FieldPtrs fp,
                                                         uint32_t* __restrict__ flags4) {
  const int nq = g.n[0] / 4;
  const int q = blockIdx.x * 64 + threadIdx.x, y = blockIdx.y * 4 + threadIdx.y;
  const int z = blockIdx.z;
  if (q >= nq || y >= g.n[1]) return;
  flags4[nq * (y + g.n[1] * z) + q] = quad_flag_bits<D, T>(g, fp, q, y, z);
}

__global__ __launch_bounds__(256) void window_x_quad_kernel(GridArgs g,
                                                            const uint32_t* __restrict__ flags4,
                                                            unsigned long long* __restrict__ out4) {
  const int nq = g.n[0] / 4;
  const int q = blockIdx.x * 64 + threadIdx.x, y = blockIdx.y * 4 + threadIdx.y;
  const int z = blockIdx.z;
  if (q >= nq || y >= g.n[1]) return;
  const int rowq = nq * (y + g.n[1] * z);
  // nq >= 2 since n0 >= 6.
  out4[rowq + q] = quad_window_x(flags4[rowq + (q == 0 ? nq - 1 : q - 1)], flags4[rowq + q],
                                 flags4[rowq + (q + 1 == nq ? 0 : q + 1)]);
}

// The y and z window passes of a 3-D grid in one: the low bytes OR over the
// 6 x 6 (y, z) block y-2..y+3, z-2..z+3 of the x-window words and the high
// bytes over the 4 x 4 block y-1..y+2, z-1..z+2 (the two separable passes
// composed).  A 64 x 4 workgroup owns 64 quads x 4 rows and marches through
// kZChunk planes: each plane's rows y0-2..y0+6 go through LDS (two buffers,
// one barrier per plane), each work-item forms its y window and keeps the
// last six in registers for the z window.  The rows are loaded kZAhead planes
// ahead into registers, so that loads stay in flight across the planes.
// Every input word is read from memory once per chunk (plus the 5-plane
// halo), every output written once.
// Grid: (ceil(nq / 64), ceil(n1 / 4), ceil(n2 / kZChunk)) of 64 x 4.
constexpr int kZChunk = 32;
constexpr int kZAhead = 4;
__global__ __launch_bounds__(256) void window_yz3_quad_kernel(
    GridArgs g, const unsigned long long* __restrict__ in4, unsigned long long* __restrict__ out4) {
  constexpr unsigned long long LO = 0x00ff00ff00ff00ffull, HI = 0xff00ff00ff00ff00ull;
  __shared__ unsigned long long s_rows[2][9][64];
  const int nq = g.n[0] / 4, n1 = g.n[1], n2 = g.n[2];
  const int tq = (int)threadIdx.x, ty = (int)threadIdx.y;
  const int q = blockIdx.x * 64 + tq;
  const int y0 = blockIdx.y * 4, y = y0 + ty;
  const int z0 = blockIdx.z * kZChunk, z1 = min(z0 + kZChunk, n2);
  const int K = z1 - z0 + 5;  // planes z0-2 .. z1+2
  const bool qok = q < nq;
  // Rows and planes wrap periodically (n1, n2 >= 6).  Work-item row ty
  // stages the LDS rows ty, ty + 4 and (ty == 0) 8.
  int roff[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    int yy = y0 - 2 + ty + 4 * i;
    yy = yy < 0 ? yy + n1 : (yy >= n1 ? yy - n1 : yy);
    roff[i] = q + nq * yy;
  }
  const int nrow = ty == 0 ? 3 : 2;
  int zl = z0 - 2 < 0 ? z0 - 2 + n2 : z0 - 2;  // plane of the next load
  unsigned long long pre[kZAhead][3];
  const auto load_plane = [&](unsigned long long* r) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
      r[i] = qok && i < nrow ? in4[roff[i] + nq * n1 * zl] : 0ull;
    zl = zl + 1 == n2 ? 0 : zl + 1;
  };
#pragma unroll
  for (int j = 0; j < kZAhead; ++j)
    if (j < K) load_plane(pre[j]);
  unsigned long long lo[6] = {0, 0, 0, 0, 0, 0}, hi[6] = {0, 0, 0, 0, 0, 0};
  for (int k0 = 0; k0 < K; k0 += kZAhead) {
#pragma unroll
    for (int j = 0; j < kZAhead; ++j) {
      const int k = k0 + j;
      if (k >= K) break;  // uniform over the workgroup
      const int buf = k & 1;
#pragma unroll
      for (int i = 0; i < 3; ++i)
        if (i < nrow) s_rows[buf][ty + 4 * i][tq] = pre[j][i];
      __syncthreads();
      if (k + kZAhead < K) load_plane(pre[j]);
      unsigned long long l = 0, h = 0;
#pragma unroll
      for (int d = 0; d < 6; ++d) {
        const unsigned long long v = s_rows[buf][ty + d][tq];
        l |= v & LO;
        if (d >= 1 && d <= 4) h |= v & HI;
      }
#pragma unroll
      for (int m = 0; m < 5; ++m) {
        lo[m] = lo[m + 1];
        hi[m] = hi[m + 1];
      }
      lo[5] = l;
      hi[5] = h;
      if (k >= 5 && qok && y < n1) {
        const int zo = z0 + k - 5;
        out4[q + nq * (y + n1 * zo)] =
            (lo[0] | lo[1] | lo[2] | lo[3] | lo[4] | lo[5]) | (hi[1] | hi[2] | hi[3] | hi[4]);
      }
    }
  }
}

}  // namespace sl
