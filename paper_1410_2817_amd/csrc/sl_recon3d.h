// 3-D reconstruction for gfx950 (Sec. 2.1-2.3).
//
// The limiter's order choice for a node depends only on its host cell r: the
// quintic stencil reads the jump flags of the 6^3 nodes r-2..r+3 and the cubic
// one those of the 4^3 nodes r-1..r+2.  Both ORs are separable, so three short
// passes (x, y, z) turn the per-node flag bytes into one 16-bit word per cell
// (low byte: quintic window, high byte: cubic window, bit f for field f), and
// the reconstruction reads a single word per node instead of 216 flag bytes.
//
// The reconstruction kernel gives each workgroup a TX x TY x TZ tile of mesh
// nodes (one per work-item, one z-plane of TX x TY per wave), tiles assigned
// XCD by XCD so that neighbouring tiles share an L2.  Every node runs the
// fixed-iteration Newton on its start cell, the full walk if that fails,
// reads its order word, and evaluates the separable Z-spline sum.  When no
// stencil of the wave wraps around the periodic box, the 216 taps are buffer
// loads whose per-row offsets are wave-uniform (scalar registers) and whose
// six x-taps are contiguous, so the compiler issues them as a few wide loads
// with no per-tap address arithmetic; otherwise the taps go through wrapped
// index tables.  Both paths sum in the same order.
#pragma once

#include "sl_orders.h"
#include "sl_recon2d.h"

namespace sl {

// Lattice displacement through the caches.
struct NearDisp3D {
  const double* __restrict__ gdisp;
  GridArgs g;
  __device__ __forceinline__ void operator()(const int* v, double* d) const {
    const int lin = wrap_near(v[0], g.n[0]) +
                    g.n[0] * (wrap_near(v[1], g.n[1]) + g.n[1] * wrap_near(v[2], g.n[2]));
    d[0] = gdisp[lin];
    d[1] = gdisp[(size_t)g.ntot + lin];
    d[2] = gdisp[2 * (size_t)g.ntot + lin];
  }
};

struct Tile3D {
  static constexpr int TX = 8;
  static constexpr int TY = 8;
  static constexpr int TZ = 4;
};
static_assert(Tile3D::TX * Tile3D::TY * Tile3D::TZ == kTileThreads, "one node per work-item");

// Raw buffer loads: the descriptor covers one field, offsets are in bytes.
// The fourth descriptor word is the gfx9 data format for 32-bit elements.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t field_rsrc(const void* p, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, bytes, 0x00020000);
}

template <typename T>
__device__ __forceinline__ T buffer_value(__amdgpu_buffer_rsrc_t rs, int voff, int soff);

template <>
__device__ __forceinline__ float buffer_value<float>(__amdgpu_buffer_rsrc_t rs, int voff,
                                                     int soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, voff, soff, 0));
}

template <>
__device__ __forceinline__ double buffer_value<double>(__amdgpu_buffer_rsrc_t rs, int voff,
                                                       int soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0));
}

// Separable 6x6x6 Z-spline sum; val(kx, ky, kz) is the value of node
// r - 2 + (kx, ky, kz).  x innermost, then y, then z, on every path.  The z
// loop stays rolled: unrolled (on the LDS path) the hoisted loads spilled
// registers, 7.97 -> 9.77 ms per deformational 512^3 FP64 launch and 6.87 ->
// 7.49 ms in FP32.  Each plane reads its rows in pairs, the twelve values
// before their products, so that a wave keeps six LDS reads in flight: with
// one row sum fed straight from the reads the schedule waited on every read
// (deformational 512^3 FP64 step 7.60 -> 7.56 ms, Fourier 256^3 1.91 ->
// 1.75 ms).  FENCE keeps the compiler from moving a pair's reads into the
// products (one-field kernels: FP64 7.56 -> 7.47 ms, FP32 values 6.28 -> 6.23
// ms; three Fourier fields lose 2 %, so they go without).  The z weights
// shift down one slot per plane (a rolled loop cannot index a register array
// without scratch memory or a chain of selects).  Same operation order as the
// plain triple loop, so the value is bitwise that of the other paths.
template <bool FENCE, typename T, class Val>
__device__ __forceinline__ T zsum3d(const T* wx, const T* wy, const T* wz, const Val& val) {
  T acc = T(0);
  T w0 = wz[0], w1 = wz[1], w2 = wz[2], w3 = wz[3], w4 = wz[4], w5 = wz[5];
#pragma unroll 1
  for (int kz = 0; kz < 6; ++kz) {
    T pl = T(0);
#pragma unroll
    for (int ky = 0; ky < 6; ky += 2) {
      T v[2][6];
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int kx = 0; kx < 6; ++kx) v[r][kx] = val(kx, ky + r, kz);
      if constexpr (FENCE) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        T s = T(0);
#pragma unroll
        for (int kx = 0; kx < 6; ++kx) s = fma(v[r][kx], wx[kx], s);
        pl = fma(s, wy[ky + r], pl);
      }
    }
    acc = fma(pl, w0, acc);
    w0 = w1;
    w1 = w2;
    w2 = w3;
    w3 = w4;
    w4 = w5;
  }
  return acc;
}

// The linear (Z0) sum: only taps 2..3 of each axis carry weight, so this
// 2 x 2 x 2 sum in the same order equals zsum3d on finite values (each
// skipped term adds an exact zero).  Taken where a whole wave is at order 0.
template <typename T, class Val>
__device__ __forceinline__ T zsum3d_linear(const T* wx, const T* wy, const T* wz,
                                           const Val& val) {
  T acc = T(0);
#pragma unroll
  for (int kz = 2; kz <= 3; ++kz) {
    T pl = T(0);
#pragma unroll
    for (int ky = 2; ky <= 3; ++ky) {
      T s = T(0);
#pragma unroll
      for (int kx = 2; kx <= 3; ++kx) s = fma(val(kx, ky, kz), wx[kx], s);
      pl = fma(s, wy[ky], pl);
    }
    acc = fma(pl, wz[kz], acc);
  }
  return acc;
}

// LDS box of field values for one tile: the tile, the quintic stencil (5),
// one cell of walk margin on each side and one of spread in the start cells.
// Boxes of more than 48 KB (many fields, or FP64 with more than one field)
// are not staged; their taps are read through the caches.  Reading every tap
// through the caches measured 2x slower on the deformational flow (8.3 ->
// 16.5 ms per 512^3 launch) and 3x on the Fourier flow (2.0 -> 6.0 ms per
// 256^3 launch).
template <typename T, int NF>
struct Box3D {
  static constexpr int BX = Tile3D::TX + 8;
  static constexpr int BY = Tile3D::TY + 8;
  static constexpr int BZ = Tile3D::TZ + 8;
  static constexpr int bytes(int px) { return NF * (int)sizeof(T) * px * BY * BZ; }
  // LDS row pitch: a wave's 8 x 8 lanes read 8 consecutive x values in each
  // of 8 rows; a pitch of 24 elements (8 mod 16) puts the rows of each
  // half-wave on distinct LDS banks for 4- and 8-byte values alike.  Boxes
  // that would then no longer fit four workgroups per CU keep the unpadded
  // pitch (occupancy matters more there than the bank conflicts).
  static constexpr int PX = bytes(BX + 8) <= 40 * 1024 ? BX + 8 : BX;
  static constexpr int NB = PX * BY * BZ;  // elements per field
  static constexpr bool STAGE = bytes(PX) <= 48 * 1024;
  // Waves per SIMD the register budget targets: four workgroups per CU when
  // their boxes fit 160 KB of LDS, three otherwise.
  static constexpr int WAVES = STAGE && bytes(PX) <= 40 * 1024 ? 4 : 3;
};

// Element solve in cell r for the search.  When no active lane's cell
// touches the periodic seam the eight vertex displacements are buffer loads at
// wave-uniform offsets from the cell's lower vertex (x pairs are adjacent);
// otherwise they go through the wrapped accessor.  Same code as
// element_solve<3>.
__device__ __forceinline__ int cell_solve3d(const GridArgs& g, const double* __restrict__ gdisp,
                                            const NearDisp3D& acc, int dbuf_ok, const int* tgt,
                                            const int* r, double* xi) {
  bool seam = false;
#pragma unroll
  for (int a = 0; a < 3; ++a) seam = seam || r[a] < 0 || r[a] + 1 >= g.n[a];
  double V[8][3];
  if (dbuf_ok && __ballot(seam) == 0ull) {
    const int sy = g.n[0], sz = g.n[0] * g.n[1];
    const int vb = (r[0] + sy * r[1] + sz * r[2]) * 8;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const __amdgpu_buffer_rsrc_t rs = field_rsrc(gdisp + (size_t)a * g.ntot, g.ntot * 8);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int ex = e & 1, ey = (e >> 1) & 1, ez = e >> 2;
        const double d = buffer_value<double>(rs, vb + 8 * ex, 8 * (ey * sy + ez * sz));
        V[e][a] = (double)(r[a] + ((e >> a) & 1) - tgt[a]) + d;
      }
    }
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      int v[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) v[a] = r[a] + ((e >> a) & 1);
      double d[3];
      acc(v, d);
#pragma unroll
      for (int a = 0; a < 3; ++a) V[e][a] = (double)(v[a] - tgt[a]) + d[a];
    }
  }
  Element<3> el;
  el.set(V);
  return el.solve(g, xi);
}

// The next step's trajectory of lattice node tgt (a fresh lattice): family VK,
// or the grid's family at run time when VK < 0.
template <int VK>
__device__ __forceinline__ void next_traj3d(const GridArgs& g, const VelArgs& v,
                                            const NextTraj& nt, const int* tgt) {
  if constexpr (VK < 0)
    traj_any<3>(g, v, nt.disp, nt.st, nt.dt, nt.integrator, tgt, nt.trig);
  else
    traj_node<3, VK>(g, v, nt.disp, nt.st, nt.dt, 0, nt.integrator, tgt, nt.trig);
}

// `ord` holds the window words (null when the limiter is off); `buf_ok` is
// non-zero when one field's bytes fit the 31-bit buffer offsets, `dbuf_ok`
// when one displacement component's do; `nt` / `v`: the next step's
// trajectories of the tile's nodes (NextTraj).
// VK: the velocity family of the fused next-step trajectories when the kernel
// is specialised for one (the deformational flow with one field, whose
// registers then need not cover every family's), or -1 for the run-time
// switch over all of them.
template <typename T, int NF, int VK = -1>
__global__ __launch_bounds__(kTileThreads, (Box3D<T, NF>::WAVES)) void recon3d_kernel(
    GridArgs g, FieldPtrs fp, const double* __restrict__ gdisp,
    const uint16_t* __restrict__ ord, unsigned long long* __restrict__ stats, int tiles_x,
    int tiles_y, int ntiles, int buf_ok, int dbuf_ok, NextTraj nt, VelArgs v) {
  using C = Tile3D;
  using X = Box3D<T, NF>;
  constexpr int nf = NF;
  __shared__ unsigned s_cnt[ST_COUNT];
  __shared__ int s_min[3];
  __shared__ T lval[X::STAGE ? nf * X::NB : 1];
  if (threadIdx.x < ST_COUNT) s_cnt[threadIdx.x] = 0u;
  if (threadIdx.x < 3) s_min[threadIdx.x] = INT_MAX;
  __syncthreads();

  const int tile = xcd_tile(blockIdx.x, ntiles);
  const int tx = tile % tiles_x, rest = tile / tiles_x;
  const int ty = rest % tiles_y, tz = rest / tiles_y;
  const int x = tx * C::TX + (int)threadIdx.x % C::TX;
  const int y = ty * C::TY + ((int)threadIdx.x / C::TX) % C::TY;
  const int z = tz * C::TZ + (int)threadIdx.x / (C::TX * C::TY);
  const bool act = x < g.n[0] && y < g.n[1] && z < g.n[2];
  const int sy = g.n[0], sz = g.n[0] * g.n[1];
  const int lin = x + sy * y + sz * z;
  const int tgt[3] = {x, y, z};

  // The next step's trajectory of this work-item's lattice node (NextTraj);
  // it touches nothing the reconstruction below reads.  Where a work-item's
  // share of the box fits 24 registers, the box loads are issued first and
  // stay in flight while it integrates (OVERLAP: deformational 512^3 step
  // 8.65 -> 8.55 ms in FP64, 7.33 -> 7.23 ms with FP32 values); otherwise it
  // integrates first.
  constexpr bool OVERLAP = X::STAGE && X::BZ * nf * (int)sizeof(T) <= 96;
  if constexpr (!OVERLAP) {
    if (nt.disp && !nt.carried && act)
      next_traj3d<VK>(g, v, nt, tgt);
  }

  // 1. Own displacement and start cell.
  double d0[3] = {0.0, 0.0, 0.0};
  int r[3] = {0, 0, 0};
  if (act) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      d0[a] = gdisp[(size_t)a * g.ntot + lin];
      r[a] = (int)floor((double)tgt[a] - d0[a]);
    }
  }
  // 2. Stage the values of the box at the tile's lowest start cell.
  int ox[3] = {0, 0, 0};
  if constexpr (X::STAGE) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int m = wave_min(act ? r[a] : INT_MAX);
      if (__lane_id() == 0) atomicMin(&s_min[a], m);
    }
    __syncthreads();
    // Clamped so that garbage start cells cannot overflow the box origin.
#pragma unroll
    for (int a = 0; a < 3; ++a) ox[a] = max(s_min[a], -(1 << 28)) - 3;
    // Work-item t stages the z-column (t % BX, t / BX) of the box: one
    // wrapped x/y offset per work-item, then BZ loads stepping in z.
    static_assert(X::BX * X::BY == kTileThreads, "one box column per work-item");
    const int bx = (int)threadIdx.x % X::BX, by = (int)threadIdx.x / X::BX;
    const int gxy = wrap_near(ox[0] + bx, g.n[0]) + sy * wrap_near(ox[1] + by, g.n[1]);
    int gz = wrap_near(ox[2], g.n[2]);
    if constexpr (OVERLAP && VK >= 0) {
      // The trajectory's own loads (its evaluator's sin/cos table) go out
      // before the box loads: loads complete in issue order, so issued after
      // them they made the trajectory wait for the whole box.
      const bool traj = nt.disp && !nt.carried && act;
      NodeVelocity<VK, 3> vel{};
      double td[3], tx[3];
      if (traj) traj_start<3>(g, v, vel, nt.disp, nt.dt, 0, tgt, nt.trig, td, tx);
      T sv[X::BZ][nf];
#pragma unroll
      for (int bz = 0; bz < X::BZ; ++bz) {
        const int gl = gxy + sz * gz;
#pragma unroll
        for (int f = 0; f < nf; ++f) sv[bz][f] = static_cast<const T*>(fp.in[f])[gl];
        gz = gz + 1 == g.n[2] ? 0 : gz + 1;
      }
      if (traj) traj_finish<3>(g, v, vel, nt.disp, nt.st, nt.dt, nt.integrator, tgt, td, tx);
#pragma unroll
      for (int bz = 0; bz < X::BZ; ++bz)
#pragma unroll
        for (int f = 0; f < nf; ++f)
          lval[f * X::NB + bx + X::PX * by + X::PX * X::BY * bz] = sv[bz][f];
    } else if constexpr (OVERLAP) {
      T sv[X::BZ][nf];
#pragma unroll
      for (int bz = 0; bz < X::BZ; ++bz) {
        const int gl = gxy + sz * gz;
#pragma unroll
        for (int f = 0; f < nf; ++f) sv[bz][f] = static_cast<const T*>(fp.in[f])[gl];
        gz = gz + 1 == g.n[2] ? 0 : gz + 1;
      }
      if (nt.disp && !nt.carried && act)
        next_traj3d<VK>(g, v, nt, tgt);
#pragma unroll
      for (int bz = 0; bz < X::BZ; ++bz)
#pragma unroll
        for (int f = 0; f < nf; ++f)
          lval[f * X::NB + bx + X::PX * by + X::PX * X::BY * bz] = sv[bz][f];
    } else {
#pragma unroll 4
      for (int bz = 0; bz < X::BZ; ++bz) {
        const int gl = gxy + sz * gz;
#pragma unroll
        for (int f = 0; f < nf; ++f)
          lval[f * X::NB + bx + X::PX * by + X::PX * X::BY * bz] =
              static_cast<const T*>(fp.in[f])[gl];
        gz = gz + 1 == g.n[2] ? 0 : gz + 1;
      }
    }
    __syncthreads();
  }

  int walked_any = 0, scanned_any = 0, sfail = 0, nfail = 0, c0 = 0, c1 = 0, c2 = 0, bad = 0;
  if (act) {
    const NearDisp3D acc{gdisp, g};
    double xi[3];
    int walked = 0, loc = LOC_OK;
    const auto solve = [&](const int* rr, double* xx) {
      return cell_solve3d(g, gdisp, acc, dbuf_ok, tgt, rr, xx);
    };
    const int rc0 = solve(r, xi);
    if (rc0 != 1 || !in_cube<3>(g, xi)) {
      const double x0[3] = {xi[0], xi[1], xi[2]};
      loc = locate_from<3>(g, solve, rc0, x0, r, xi, walked);
    }
    walked_any = walked != 0;
    scanned_any = walked == 2;
    if (loc != LOC_OK) {
      sfail = loc == LOC_SEARCH_FAIL;
      nfail = loc == LOC_NEWTON_FAIL;
#pragma unroll
      for (int f = 0; f < nf; ++f) static_cast<T*>(fp.out[f])[lin] = T(NAN);
      if (nt.carried && nt.disp)
        for (int a = 0; a < 3; ++a) nt.disp[(size_t)a * g.ntot + lin] = NAN;
    } else {

      int w0[3], lb[3];
      bool interior = true, inbox = X::STAGE;
      constexpr int B[3] = {X::BX, X::BY, X::BZ};
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        interior = interior && r[a] - 2 >= 0 && r[a] + 3 < g.n[a];
        w0[a] = wrap_near(r[a], g.n[a]);
        lb[a] = r[a] - 2 - ox[a];
        inbox = inbox && (unsigned)lb[a] <= (unsigned)(B[a] - 6);
      }
      const int lbase = lb[0] + X::PX * (lb[1] + X::BY * lb[2]);
      const bool lim = g.limiter && g.order_max > 0;
      unsigned or6 = 0, or4 = 0;
      if (lim) {
        const unsigned o = ord[w0[0] + sy * w0[1] + sz * w0[2]];
        or6 = o & 0xffu;
        or4 = o >> 8;
      }
      // Lanes outside the box read through the caches: with buffer loads
      // when none of them wraps around the periodic box.
      const bool fast = buf_ok && __ballot(!inbox && !interior) == 0ull;
      int ix[6], iy[6], iz[6];
      int vbase = 0;
      if (!inbox) {
        if (fast) {
          vbase = ((r[0] - 2) + sy * (r[1] - 2) + sz * (r[2] - 2)) * (int)sizeof(T);
        } else {
          int wx = wrap_near(r[0] - 2, g.n[0]), wy = wrap_near(r[1] - 2, g.n[1]),
              wz = wrap_near(r[2] - 2, g.n[2]);
#pragma unroll
          for (int s = 0; s < 6; ++s) {
            ix[s] = wx;
            iy[s] = sy * wy;
            iz[s] = sz * wz;
            wx = wx + 1 == g.n[0] ? 0 : wx + 1;
            wy = wy + 1 == g.n[1] ? 0 : wy + 1;
            wz = wz + 1 == g.n[2] ? 0 : wz + 1;
          }
        }
      }
      const int fbytes = buf_ok ? g.ntot * (int)sizeof(T) : 0;
      const T t[3] = {(T)xi[0], (T)xi[1], (T)xi[2]};
      // linear_c: std::true_type for the 2 x 2 x 2 sum of a wave that is at
      // order 0 throughout, std::false_type for the full sum.
      auto field_value = [&](int f, const T* wx, const T* wy, const T* wz, auto linear_c) {
        const auto sum = [&](const auto& at) {
          if constexpr (decltype(linear_c)::value) return zsum3d_linear<T>(wx, wy, wz, at);
          else return zsum3d<NF == 1, T>(wx, wy, wz, at);
        };
        T v;
        if (inbox) {
          const T* lv = lval + f * X::NB + lbase;
          v = sum([&](int kx, int ky, int kz) { return lv[kx + X::PX * (ky + X::BY * kz)]; });
        } else if (fast) {
          const __amdgpu_buffer_rsrc_t rs = field_rsrc(fp.in[f], fbytes);
          v = sum([&](int kx, int ky, int kz) {
            return buffer_value<T>(rs, vbase + kx * (int)sizeof(T),
                                   (kz * sz + ky * sy) * (int)sizeof(T));
          });
        } else {
          const T* __restrict__ h = static_cast<const T*>(fp.in[f]);
          v = sum([&](int kx, int ky, int kz) { return h[ix[kx] + iy[ky] + iz[kz]]; });
        }
        bad += !isfinite(v);
        static_cast<T*>(fp.out[f])[lin] = v;
        // Carried velocity: fields 0..2 give the next step's displacement
        // (the spacing by selects: the field index may be a loop variable).
        if (f < 3 && nt.carried && nt.disp) {
          const double hf = f == 0 ? g.h[0] : (f == 1 ? g.h[1] : g.h[2]);
          nt.disp[(size_t)f * g.ntot + lin] = nt.dt * (double)v / hf;
        }
      };
      const unsigned fmask = nf >= 32 ? 0xffffffffu : ((1u << nf) - 1u);
      const bool low = lim && (((or6 | or4) & fmask) != 0u);
      if (__ballot(low) == 0ull) {
        c0 += g.order_max == 0 ? nf : 0;
        c1 += g.order_max == 1 ? nf : 0;
        c2 += g.order_max == 2 ? nf : 0;
        T w[3][6];
#pragma unroll
        for (int a = 0; a < 3; ++a) zspline_weights<T>(g.order_max, t[a], w[a]);
#pragma unroll
        for (int f = 0; f < nf; ++f) field_value(f, w[0], w[1], w[2], std::false_type{});
      } else {
        // Some lane of the wave drops an order: weights per field and lane;
        // a field the whole wave takes at linear order sums its 8 taps only
        // (flags cover regions, so this is the usual lowered case).
#pragma unroll 1
        for (int f = 0; f < nf; ++f) {
          const int m = pick_order(g.order_max, or6, or4, f);
          c0 += m == 0;
          c1 += m == 1;
          c2 += m == 2;
          T w[3][6];
#pragma unroll
          for (int a = 0; a < 3; ++a) zspline_weights<T>(m, t[a], w[a]);
          if (__ballot(m != 0) == 0ull)
            field_value(f, w[0], w[1], w[2], std::true_type{});
          else
            field_value(f, w[0], w[1], w[2], std::false_type{});
        }
      }
    }
  }
  // Counters: per-wave sums packed 16 + 16 bits (at most 64 * 8 per wave),
  // one LDS atomic per wave, one global atomic per workgroup and counter.
  const unsigned p0 = wave_sum((unsigned)walked_any | ((unsigned)scanned_any << 16));
  const unsigned p1 = wave_sum((unsigned)sfail | ((unsigned)nfail << 16));
  // Order counts per wave fit 10 bits each (at most 64 lanes x 8 fields).
  const unsigned p2 = wave_sum((unsigned)c0 | ((unsigned)c1 << 10) | ((unsigned)c2 << 20));
  const unsigned p3 = wave_sum((unsigned)bad);
  if (__lane_id() == 0) {
    if (p0 & 0xffffu) atomicAdd(&s_cnt[ST_WALKED], p0 & 0xffffu);
    if (p0 >> 16) atomicAdd(&s_cnt[ST_SCANNED], p0 >> 16);
    if (p1 & 0xffffu) atomicAdd(&s_cnt[ST_SEARCH_FAIL], p1 & 0xffffu);
    if (p1 >> 16) atomicAdd(&s_cnt[ST_NEWTON_FAIL], p1 >> 16);
    if (p2 & 0x3ffu) atomicAdd(&s_cnt[ST_ORDER0], p2 & 0x3ffu);
    if ((p2 >> 10) & 0x3ffu) atomicAdd(&s_cnt[ST_ORDER1], (p2 >> 10) & 0x3ffu);
    if (p2 >> 20) atomicAdd(&s_cnt[ST_ORDER2], p2 >> 20);
    if (p3) atomicAdd(&s_cnt[ST_NONFINITE], p3);
  }
  __syncthreads();
  if (threadIdx.x < ST_COUNT && s_cnt[threadIdx.x])
    atomicAdd(stat_copy(stats) + threadIdx.x, (unsigned long long)s_cnt[threadIdx.x]);
}

}  // namespace sl
