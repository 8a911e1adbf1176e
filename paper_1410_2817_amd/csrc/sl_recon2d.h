// Tiled 2-D reconstruction kernel for gfx950 (Sec. 2.1-2.3).
//
// A workgroup of 256 work-items owns a TX x TY tile of mesh nodes.  It reads
// the displacement of its own nodes (the start guesses of the element walk),
// reduces their departure cells to a bounding box, and stages into LDS the
// field values of that box (plus a margin for the walk) grown by one node
// (the jump criterion needs neighbours).  The element solves read the
// vertex displacements through the caches: staging them in LDS as well
// measured slower (51.4 -> 54.5 us per 1024^2 launch, 0.608 -> 0.639 ms at
// 4096^2), the loads being few and the L1/L2 hit rate high.
// The jump flags of the box are computed once from the staged values and
// OR-reduced over the quintic and cubic stencil windows by separable passes,
// so each node reads its order mask with two LDS loads.  Every node then runs
// the walk + Newton, picks its order per field and evaluates the separable
// Z-spline sum from LDS.  A node whose walk leaves the staged box (or a tile
// whose box does not fit in LDS) takes the same arithmetic through global
// memory, so the result does not depend on the path.
//
// Tiles are assigned XCD by XCD: consecutive workgroups are dispatched
// round-robin over the 8 XCDs, and the mapping below gives each XCD a
// contiguous run of tiles so that neighbouring halos meet in the same L2.
#pragma once

#include <type_traits>

#include "sl_device.h"
#include "sl_traj.h"

namespace sl {

constexpr int kTileThreads = 256;
constexpr int kWalkMargin = 1;   // extra cells staged around the start cells
constexpr int kNumXcd = 8;

// 16 x 16 tiles, one mesh node per work-item: small LDS boxes and few live
// registers keep four workgroups resident per CU, which hides the latency of
// the staging loads behind other workgroups' arithmetic.
template <typename T, int NF>
struct Tile2D {
  static constexpr int TX = 16;
  static constexpr int TY = 16;
  static constexpr int NPT = TX * TY / kTileThreads;  // nodes per work-item
  // Dynamic LDS sized for a departure box of up to BOX x BOX nodes (the tile,
  // the quintic stencil, the walk margin and a few cells of spread in the
  // start cells); larger boxes take the global path.  Keeping the allocation
  // tight lets many workgroups share a CU's 160 KB.
  static constexpr int BOX = TX + 5 + 2 * kWalkMargin + 3;
  static constexpr int RAW = (BOX + 2) * (BOX + 2) * NF * (int)sizeof(T) + NF * BOX * 4 + 64;
  static constexpr int CAP = 60 * 1024;  // stay under the 64 KB workgroup limit
  static constexpr int LDS_BYTES = (RAW + 255) / 256 * 256 < CAP ? (RAW + 255) / 256 * 256 : CAP;
};

// Waves per SIMD the register budget of the 2-D reconstruction kernels
// targets, per (precision, field count, velocity family VK of a specialised
// kernel): the most that compile without spills (the LDS boxes allow more),
// except where more waves with spills measured faster: FP64 with two fields
// at four waves spills 20 VGPRs (Burgers 512^2 step 18.0 -> 15.7 us), and a
// carried velocity with three FP64 fields, whose kernel integrates no
// trajectories, at five waves (Kelvin 1024^2 reconstruction 35.8 -> 33.9 us;
// with the fused trajectories five waves lost 18 %).
template <typename T, int NF, int VK = -1>
constexpr int tile2d_waves() {
  if (sizeof(T) == 4) return (NF >= 2 && NF <= 4) ? 6 : (NF == 1 ? 5 : 4);
  if (NF == 3 && VK == SL_VEL_CARRIED) return 5;
  return NF <= 3 ? 4 : 3;
}

__device__ __forceinline__ int xcd_tile(int b, int nblocks) {
  const int xcd = b % kNumXcd, local = b / kNumXcd;
  const int q = nblocks / kNumXcd, rem = nblocks % kNumXcd;
  return xcd * q + (xcd < rem ? xcd : rem) + local;
}

// Displacement accessor reading global memory (through L1/L2).
struct NearDisp2D {
  const double* __restrict__ gdisp;
  GridArgs g;
  __device__ __forceinline__ void operator()(const int* v, double* d) const {
    const int lin = wrap_near(v[0], g.n[0]) + g.n[0] * wrap_near(v[1], g.n[1]);
    d[0] = gdisp[lin];
    d[1] = gdisp[(size_t)g.ntot + lin];
  }
};

// Element solve in cell r with the global accessor: the four vertex indices
// from one wrap per axis.  Same values and arithmetic as element_solve<2>.
__device__ __forceinline__ int element_solve_near(const GridArgs& g, const NearDisp2D& acc,
                                                  const int* tgt, const int* r, double* xi) {
  const int x0 = wrap_near(r[0], g.n[0]), y0 = wrap_near(r[1], g.n[1]);
  const int x1 = x0 + 1 == g.n[0] ? 0 : x0 + 1, y1 = y0 + 1 == g.n[1] ? 0 : y0 + 1;
  const int row0 = g.n[0] * y0, row1 = g.n[0] * y1;
  const int lin[4] = {x0 + row0, x1 + row0, x0 + row1, x1 + row1};
  const double* __restrict__ gy = acc.gdisp + (size_t)g.ntot;
  double V[4][2];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    V[e][0] = (double)(r[0] + (e & 1) - tgt[0]) + acc.gdisp[lin[e]];
    V[e][1] = (double)(r[1] + (e >> 1) - tgt[1]) + gy[lin[e]];
  }
  Element<2> el;
  el.set(V);
  return el.solve(g, xi);
}

// The eight displacement values of cell r's vertices (x then y per vertex),
// and the solve from them: the same values and arithmetic as
// element_solve_near, with the loads issued early by the caller.
__device__ __forceinline__ void cell_disp_near(const GridArgs& g, const NearDisp2D& acc,
                                               const int* r, double* vd) {
  const int x0 = wrap_near(r[0], g.n[0]), y0 = wrap_near(r[1], g.n[1]);
  const int x1 = x0 + 1 == g.n[0] ? 0 : x0 + 1, y1 = y0 + 1 == g.n[1] ? 0 : y0 + 1;
  const int row0 = g.n[0] * y0, row1 = g.n[0] * y1;
  const int lin[4] = {x0 + row0, x1 + row0, x0 + row1, x1 + row1};
  const double* __restrict__ gy = acc.gdisp + (size_t)g.ntot;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    vd[2 * e] = acc.gdisp[lin[e]];
    vd[2 * e + 1] = gy[lin[e]];
  }
}

__device__ __forceinline__ int element_solve_pre(const GridArgs& g, const int* tgt, const int* r,
                                                 const double* vd, double* xi) {
  double V[4][2];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    V[e][0] = (double)(r[0] + (e & 1) - tgt[0]) + vd[2 * e];
    V[e][1] = (double)(r[1] + (e >> 1) - tgt[1]) + vd[2 * e + 1];
  }
  Element<2> el;
  el.set(V);
  return el.solve(g, xi);
}

// Jump-flag bits (all fields) of the lattice node at wrapped (x, y), from
// global memory.
template <typename T, int NF>
__device__ __forceinline__ unsigned global_flag_bits(const GridArgs& g, const FieldPtrs& fp,
                                                     int x, int y) {
  const int xm = x == 0 ? g.n[0] - 1 : x - 1, xp = x + 1 == g.n[0] ? 0 : x + 1;
  const int ym = y == 0 ? g.n[1] - 1 : y - 1, yp = y + 1 == g.n[1] ? 0 : y + 1;
  unsigned bits = 0;
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    const T* __restrict__ h = static_cast<const T*>(fp.in[f]);
    const double hc = (double)h[x + g.n[0] * y];
    const bool fl = jump_flag((double)h[xm + g.n[0] * y], hc, (double)h[xp + g.n[0] * y], g.theta) ||
                    jump_flag((double)h[x + g.n[0] * ym], hc, (double)h[x + g.n[0] * yp], g.theta);
    bits |= (fl ? 1u : 0u) << f;
  }
  return bits;
}

// Order of field f from the OR of the flags in its quintic / cubic stencils.
__device__ __forceinline__ int pick_order(int order_max, unsigned or6, unsigned or4, int f) {
  int m = order_max;
  if (m == 2 && ((or6 >> f) & 1u)) m = 1;
  if (m == 1 && ((or4 >> f) & 1u)) m = 0;
  return m;
}

// Wrapped stencil indices and flag masks through global memory, for nodes
// whose stencil is not in the staged box.
template <typename T, int NF>
__device__ __forceinline__ void stencil_global(const GridArgs& g, const FieldPtrs& fp,
                                                         const int* r, bool lim, int* ix,
                                                         int* iy, unsigned& or6,
                                                         unsigned& or4) {
  int wx = wrap_index(r[0] - 2, g.n[0]), wy = wrap_index(r[1] - 2, g.n[1]);
  for (int s = 0; s < 6; ++s) {
    ix[s] = wx;
    iy[s] = wy;
    wx = wx + 1 == g.n[0] ? 0 : wx + 1;
    wy = wy + 1 == g.n[1] ? 0 : wy + 1;
  }
  or6 = or4 = 0;
  if (lim) {
    for (int ky = 0; ky < 6; ++ky)
      for (int kx = 0; kx < 6; ++kx) {
        const unsigned fb = global_flag_bits<T, NF>(g, fp, ix[kx], iy[ky]);
        or6 |= fb;
        if (kx >= 1 && kx <= 4 && ky >= 1 && ky <= 4) or4 |= fb;
      }
  }
}

// Separable Z-spline sum over the 6x6 stencil; val(kx, ky) returns the value
// of node (r - 2 + kx, r - 2 + ky).  The same operation order is used on the
// LDS and the global path.
// Rows go two at a time in a rolled loop; the y weights are shifted down each
// pass so that only constant register indices occur (a rolled loop indexing
// wy[ky] would select among all six per row).
template <typename T, class Val>
__device__ __forceinline__ T zsum2d(const T* wx, const T* wy, const Val& val) {
  T acc = T(0);
  T w0 = wy[0], w1 = wy[1], w2 = wy[2], w3 = wy[3], w4 = wy[4], w5 = wy[5];
#pragma unroll 1
  for (int ky = 0; ky < 6; ky += 2) {
    T s0 = T(0), s1 = T(0);
#pragma unroll
    for (int kx = 0; kx < 6; ++kx) s0 = fma(val(kx, ky), wx[kx], s0);
#pragma unroll
    for (int kx = 0; kx < 6; ++kx) s1 = fma(val(kx, ky + 1), wx[kx], s1);
    acc = fma(s0, w0, acc);
    acc = fma(s1, w1, acc);
    w0 = w2;
    w1 = w3;
    w2 = w4;
    w3 = w5;
  }
  return acc;
}

// One workgroup's tile: the whole reconstruction of tile `tile` of a grid
// with `tiles_x` tiles per row.  NF is the number of fields (a compile-time
// constant so that the per-field loops unroll without exec-mask
// bookkeeping).  `smem` is the workgroup's dynamic LDS (Tile2D::LDS_BYTES).
//
// `ord`, when not null, holds the limiter order words of every cell (see
// sl_orders.h); the tile then skips its own flag pass and reads one word per
// node.  Otherwise the flags of the staged box are evaluated here.
//
// `nt` / `v` (VelT = VelArgs): the tile then also integrates the next step's
// trajectories of its own nodes (see NextTraj); VelT = NoVel compiles that out.
template <typename T, int NF, class VelT, int VK = -1>
__device__ __forceinline__ void recon2d_tile(const GridArgs& g, const FieldPtrs& fp,
                                             const double* __restrict__ gdisp,
                                             const uint16_t* __restrict__ ord,
                                             unsigned long long* __restrict__ stats, int tile,
                                             int tiles_x, unsigned char* smem,
                                             const NextTraj& nt, const VelT& v) {
  using C = Tile2D<T, NF>;
  __shared__ int s_box[4];  // min rx, min ry, max rx, max ry
  __shared__ unsigned s_cnt[ST_COUNT];

  const int tx0 = (tile % tiles_x) * C::TX, ty0 = (tile / tiles_x) * C::TY;
  const int lx = threadIdx.x % C::TX, ly0 = threadIdx.x / C::TX;
  constexpr int ROWS = kTileThreads / C::TX;  // rows covered per pass

  // 1a. Own displacements (start guesses), loaded before the trajectories
  // below so that their latency and that of the trajectories' table loads
  // overlap (loads complete in issue order).
  double d0[C::NPT][2];
  bool act[C::NPT];
#pragma unroll
  for (int k = 0; k < C::NPT; ++k) {
    const int x = tx0 + lx, y = ty0 + ly0 + ROWS * k;
    act[k] = x < g.n[0] && y < g.n[1];
    d0[k][0] = d0[k][1] = 0.0;
    if (act[k]) {
      const int lin = x + g.n[0] * y;
      d0[k][0] = gdisp[lin];
      d0[k][1] = gdisp[(size_t)g.ntot + lin];
    }
  }

  // The next step's trajectories of the tile's own nodes (NextTraj); they
  // touch nothing the reconstruction below reads.
  if constexpr (std::is_same<VelT, VelArgs>::value && VK != SL_VEL_CARRIED) {
    if (nt.disp && !nt.carried) {
#pragma unroll 1
      for (int k = 0; k < C::NPT; ++k) {
        const int idx[2] = {tx0 + lx, ty0 + ly0 + ROWS * k};
        if (idx[0] < g.n[0] && idx[1] < g.n[1]) {
          // VK: the grid's velocity family when the kernel is specialised
          // for one, else the run-time switch over all of them.
          if constexpr (VK >= 0)
            traj_node<2, VK>(g, v, nt.disp, nt.st, nt.dt, 0, nt.integrator, idx, nt.trig);
          else
            traj_any<2>(g, v, nt.disp, nt.st, nt.dt, nt.integrator, idx, nt.trig);
        }
      }
    }
  }
  if (threadIdx.x == 0) {
    s_box[0] = s_box[1] = INT_MAX;
    s_box[2] = s_box[3] = INT_MIN;
  }
  if (threadIdx.x < ST_COUNT) s_cnt[threadIdx.x] = 0u;
  __syncthreads();

  // 1b. Start cells and their bounding box.
  int rs[C::NPT][2];
  int mn[2] = {INT_MAX, INT_MAX}, mx[2] = {INT_MIN, INT_MIN};
#pragma unroll
  for (int k = 0; k < C::NPT; ++k) {
    const int x = tx0 + lx, y = ty0 + ly0 + ROWS * k;
    rs[k][0] = rs[k][1] = 0;
    if (act[k]) {
      rs[k][0] = (int)floor((double)x - d0[k][0]);
      rs[k][1] = (int)floor((double)y - d0[k][1]);
      mn[0] = min(mn[0], rs[k][0]);
      mn[1] = min(mn[1], rs[k][1]);
      mx[0] = max(mx[0], rs[k][0]);
      mx[1] = max(mx[1], rs[k][1]);
    }
  }
  // The start cells' vertex displacements and, where the order words are
  // read, the start cell's word: loaded here, their latency hides behind the
  // staging and the flags.  A node whose walk leaves the start cell re-reads
  // its word below.
  const NearDisp2D acc{gdisp, g};
  double vd[C::NPT][8];
  unsigned o_start[C::NPT];
  const bool lim_words = ord != nullptr && g.limiter && g.order_max > 0;
#pragma unroll
  for (int k = 0; k < C::NPT; ++k) {
    o_start[k] = 0u;
    if (act[k]) {
      cell_disp_near(g, acc, rs[k], vd[k]);
      if (lim_words)
        o_start[k] = ord[wrap_near(rs[k][0], g.n[0]) + g.n[0] * wrap_near(rs[k][1], g.n[1])];
    }
  }
  // Wave reductions first: LDS atomics from every lane would be serialised.
  mn[0] = wave_min(mn[0]);
  mn[1] = wave_min(mn[1]);
  mx[0] = wave_max(mx[0]);
  mx[1] = wave_max(mx[1]);
  if (__lane_id() == 0) {
    atomicMin(&s_box[0], mn[0]);
    atomicMin(&s_box[1], mn[1]);
    atomicMax(&s_box[2], mx[0]);
    atomicMax(&s_box[3], mx[1]);
  }
  __syncthreads();

  // Departure box [bx0, bx0+BX) x [by0, by0+BY): every start cell's quintic
  // stencil plus the walk margin.  Values are staged one node wider.
  // Extents are formed in 64-bit and capped so that garbage displacements
  // (NaN or huge values) can only send the tile down the global path.
  const long long ex = (long long)s_box[2] - (long long)s_box[0] + 6 + 2 * kWalkMargin;
  const long long ey = (long long)s_box[3] - (long long)s_box[1] + 6 + 2 * kWalkMargin;
  const bool sane = ex > 0 && ey > 0 && ex <= 1024 && ey <= 1024;
  const int bx0 = sane ? s_box[0] - 2 - kWalkMargin : 0;
  const int by0 = sane ? s_box[1] - 2 - kWalkMargin : 0;
  const int BX = sane ? (int)ex : 0;
  const int BY = sane ? (int)ey : 0;
  const int VX = BX + 2, VY = BY + 2;
  const int nval = VX * VY;
  constexpr int nf = NF;
  // LDS layout: values (nf planes) | flag row words
  const size_t off_val = 0;
  // Jump flags are kept as one 32-bit word per field and box row (bit x set
  // when node (x, row) is flagged), so the box may be at most 32 wide.
  const size_t off_bits = off_val + (((size_t)nf * nval * sizeof(T) + 15) & ~(size_t)15);
  const size_t need = off_bits + (size_t)nf * BY * 4;
  const bool staged = sane && BX <= 32 && need <= (size_t)C::LDS_BYTES;

  T* lval = reinterpret_cast<T*>(smem + off_val);
  unsigned* lbits = reinterpret_cast<unsigned*>(smem + off_bits);  // [f][row]

  if (staged) {
    // 2. Stage the values.  Work-items cover the box as rows of
    // 32 (one wave = two rows), so no integer division is needed; wrapped
    // coordinates are advanced incrementally from the box origin.
    const int sx_lane = threadIdx.x % 32, sy_lane = threadIdx.x / 32;
    constexpr int SROWS = kTileThreads / 32;
    const int nx = g.n[0], ny = g.n[1];
    const int wx0 = wrap_index(bx0 - 1, nx), wy0 = wrap_index(by0 - 1, ny);
    const bool narrow = VX <= nx && VY <= ny;  // then one wrap suffices
    // The first column of the first MAXR rows of each work-item: all loads
    // issued before any store, so their latencies overlap (a load-store
    // loop waited on each load in turn; 4096^2 launch 0.573 -> 0.565 ms,
    // 1024^2 unchanged).  The loop below takes the rest.
    constexpr int MAXR = (C::BOX + 2 + SROWS - 1) / SROWS;
    const int batched = narrow ? sy_lane + SROWS * MAXR : 0;  // rows below: first column done
    if (narrow) {
      T sv[MAXR][nf];
      int gx = wx0 + sx_lane;
      gx = gx >= nx ? gx - nx : gx;
#pragma unroll
      for (int i = 0; i < MAXR; ++i) {
        const int vy = sy_lane + SROWS * i;
        if (vy < VY && sx_lane < VX) {
          int gy = wy0 + vy;
          gy = gy >= ny ? gy - ny : gy;
          const size_t lin = (size_t)nx * gy + gx;
#pragma unroll
          for (int f = 0; f < nf; ++f) sv[i][f] = static_cast<const T*>(fp.in[f])[lin];
        }
      }
#pragma unroll
      for (int i = 0; i < MAXR; ++i) {
        const int vy = sy_lane + SROWS * i;
        if (vy < VY && sx_lane < VX) {
#pragma unroll
          for (int f = 0; f < nf; ++f) lval[(size_t)f * nval + sx_lane + VX * vy] = sv[i][f];
        }
      }
    }
    for (int vy = sy_lane; vy < VY; vy += SROWS) {
      int gy = wy0 + vy;
      if (narrow) {
        gy = gy >= ny ? gy - ny : gy;
      } else {
        while (gy >= ny) gy -= ny;
      }
      const size_t row = (size_t)nx * gy;
      for (int vx = sx_lane + (vy < batched ? 32 : 0); vx < VX; vx += 32) {
        int gx = wx0 + vx;
        if (narrow) {
          gx = gx >= nx ? gx - nx : gx;
        } else {
          while (gx >= nx) gx -= nx;
        }
        const size_t lin = row + gx;
        const int vi = vx + VX * vy;
#pragma unroll
        for (int f = 0; f < nf; ++f)
          lval[(size_t)f * nval + vi] = static_cast<const T*>(fp.in[f])[lin];
      }
    }
    __syncthreads();
    // 3. Jump flags of the box nodes from the staged values.  Each wave takes
    // two box rows at a time (lanes 0-31 the first, 32-63 the second, lane =
    // x), evaluates the criterion in FP64 and packs the flags of each field
    // into row words with one ballot.
    if (g.limiter && g.order_max > 0 && ord == nullptr) {
      const int lane = __lane_id(), wave = threadIdx.x / 64;
      const int bx = lane & 31;
      for (int by2 = 2 * wave; by2 < BY; by2 += 2 * (kTileThreads / 64)) {
        const int by = by2 + (lane >> 5);
        const bool in = bx < BX && by < BY;
        // Idle lanes read box node (0, 0), so that every lane loads: all
        // fields' stencils are then in flight together instead of one
        // field's after another's (1024^2 step 47.0 -> 46.1 us).
        const int c = in ? (bx + 1) + VX * (by + 1) : VX + 1;
        T hs[nf][5];
#pragma unroll
        for (int f = 0; f < nf; ++f) {
          const T* lv = lval + (size_t)f * nval;
          hs[f][0] = lv[c];
          hs[f][1] = lv[c - 1];
          hs[f][2] = lv[c + 1];
          hs[f][3] = lv[c - VX];
          hs[f][4] = lv[c + VX];
        }
#pragma unroll
        for (int f = 0; f < nf; ++f) {
          // FP64 issues at the FP32 (non-packed) rate on CDNA4, so the exact
          // criterion on the stored values costs no more than a screen.
          const double hc = (double)hs[f][0];
          const bool fx = jump_flag((double)hs[f][1], hc, (double)hs[f][2], g.theta);
          const bool fy = jump_flag((double)hs[f][3], hc, (double)hs[f][4], g.theta);
          const unsigned long long m = __ballot(in && (fx || fy));
          if (lane == 0) {
            lbits[f * BY + by2] = (unsigned)m;
            if (by2 + 1 < BY) lbits[f * BY + by2 + 1] = (unsigned)(m >> 32);
          }
        }
      }
    }
    __syncthreads();
  }

  int walked_any = 0, scanned_any = 0, sfail = 0, nfail = 0, c0 = 0, c1 = 0, c2 = 0, bad = 0;

#pragma unroll 1
  for (int k = 0; k < C::NPT; ++k) {
    if (!act[k]) continue;
    const int x = tx0 + lx, y = ty0 + ly0 + ROWS * k;
    const int tgt[2] = {x, y};
    const int lin = x + g.n[0] * y;
    // Fast path: the start cell with a fixed number of Newton iterations.
    // Lanes it does not settle run the full walk (the same arithmetic).
    int r[2] = {rs[k][0], rs[k][1]};
    double xi[2];
    int walked = 0;
    int loc = LOC_OK;
    const auto solve = [&](const int* rr, double* x) {
      return element_solve_near(g, acc, tgt, rr, x);
    };
    const int rc0 = element_solve_pre(g, tgt, r, vd[k], xi);
    if (rc0 != 1 || !in_cube<2>(g, xi)) {
      const double x0[2] = {xi[0], xi[1]};
      loc = locate_from<2>(g, solve, rc0, x0, r, xi, walked);
    }
    walked_any += walked != 0;
    scanned_any += walked == 2;
    if (loc != LOC_OK) {
      sfail += loc == LOC_SEARCH_FAIL;
      nfail += loc == LOC_NEWTON_FAIL;
#pragma unroll
      for (int f = 0; f < nf; ++f) static_cast<T*>(fp.out[f])[lin] = T(NAN);
      if (nt.carried && nt.disp) {
        nt.disp[lin] = NAN;
        nt.disp[(size_t)g.ntot + lin] = NAN;
      }
      continue;
    }
    const int sx = r[0] - 2 - bx0, sy = r[1] - 2 - by0;  // stencil origin in box
    const bool inbox = staged && sx >= 0 && sy >= 0 && sx + 6 <= BX && sy + 6 <= BY;
    const bool lim = g.limiter && g.order_max > 0;
    unsigned or6 = 0, or4 = 0;
    int ix[6], iy[6];
    if (ord != nullptr) {
      if (!inbox) stencil_global<T, NF>(g, fp, r, false, ix, iy, or6, or4);
      if (lim) {
        const unsigned o =
            r[0] == rs[k][0] && r[1] == rs[k][1]
                ? o_start[k]
                : ord[wrap_near(r[0], g.n[0]) + g.n[0] * wrap_near(r[1], g.n[1])];
        or6 = o & 0xffu;
        or4 = o >> 8;
      }
    } else if (inbox) {
      if (lim) {
#pragma unroll
        for (int f = 0; f < nf; ++f) {
          const unsigned* rb = lbits + f * BY + sy;
          unsigned w6 = 0, w4 = 0;
#pragma unroll
          for (int q = 0; q < 6; ++q) {
            const unsigned row = rb[q] >> sx;  // bit j: node (sx + j, sy + q)
            w6 |= row & 0x3fu;
            if (q >= 1 && q <= 4) w4 |= row & 0x1eu;
          }
          or6 |= (w6 != 0u ? 1u : 0u) << f;
          or4 |= (w4 != 0u ? 1u : 0u) << f;
        }
      }
    } else {
      stencil_global<T, NF>(g, fp, r, lim, ix, iy, or6, or4);
    }
    // Weights of the top order; the lower orders and the per-field select
    // only run when some lane of the wave needs them (a wave-uniform branch).
    const T tx = (T)xi[0], ty = (T)xi[1];
    T w2x[6], w2y[6];
    zspline_weights<T, false>(g.order_max, tx, w2x);
    zspline_weights<T, false>(g.order_max, ty, w2y);
    const unsigned fmask = nf >= 32 ? 0xffffffffu : ((1u << nf) - 1u);
    const bool low = lim && (((or6 | or4) & fmask) != 0u);
    auto field_value = [&](int f, const T* wx, const T* wy) {
      T v;
      if (inbox) {
        const T* lv = lval + (size_t)f * nval + (sx + 1) + VX * (sy + 1);
        v = zsum2d<T>(wx, wy, [&](int kx, int ky) { return lv[kx + VX * ky]; });
      } else {
        const T* __restrict__ h = static_cast<const T*>(fp.in[f]);
        v = zsum2d<T>(wx, wy, [&](int kx, int ky) { return h[ix[kx] + g.n[0] * iy[ky]]; });
      }
      bad += !isfinite(v);
      static_cast<T*>(fp.out[f])[lin] = v;
      // Carried velocity: fields 0 and 1 give the next step's displacement.
      if (f < 2 && nt.carried && nt.disp)
        nt.disp[(size_t)f * g.ntot + lin] = nt.dt * (double)v / g.h[f];
    };
    if (__ballot(low) == 0ull) {
      c0 += g.order_max == 0 ? nf : 0;
      c1 += g.order_max == 1 ? nf : 0;
      c2 += g.order_max == 2 ? nf : 0;
#pragma unroll
      for (int f = 0; f < nf; ++f) field_value(f, w2x, w2y);
    } else {
      // A lowered order usually concerns one field of a wave: a field takes
      // the lower-order weights and the per-lane select only where some lane
      // of the wave lowers it (evaluated per such field, which keeps them
      // out of the registers live across fields).
#pragma unroll
      for (int f = 0; f < nf; ++f) {
        const int m = pick_order(g.order_max, or6, or4, f);
        c0 += m == 0;
        c1 += m == 1;
        c2 += m == 2;
        if (__ballot(m != g.order_max) == 0ull) {
          field_value(f, w2x, w2y);
          continue;
        }
        T w1x[6], w1y[6], w0x[6], w0y[6];
        zspline_weights<T, false>(g.order_max > 1 ? 1 : 0, tx, w1x);
        zspline_weights<T, false>(g.order_max > 1 ? 1 : 0, ty, w1y);
        zspline_weights<T, false>(0, tx, w0x);
        zspline_weights<T, false>(0, ty, w0y);
        const int drop = g.order_max - m;  // 0, 1 or 2 orders below the top
        T wx[6], wy[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          wx[q] = drop == 0 ? w2x[q] : (drop == 1 ? w1x[q] : w0x[q]);
          wy[q] = drop == 0 ? w2y[q] : (drop == 1 ? w1y[q] : w0y[q]);
        }
        field_value(f, wx, wy);
      }
    }
  }
  // Counters: summed in LDS, one global atomic per workgroup and counter.
  // Per-wave sums of pairs packed 16 + 16 bits (a wave's count of any of them
  // is at most 64 * 8), then one LDS atomic per wave.
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

template <typename T, int NF, int VK = -1>
__global__ __launch_bounds__(kTileThreads, (tile2d_waves<T, NF, VK>()))
void recon2d_tiled_kernel(
    GridArgs g, FieldPtrs fp, const double* __restrict__ gdisp,
    const uint16_t* __restrict__ ord, unsigned long long* __restrict__ stats, int tiles_x,
    int ntiles, NextTraj nt, VelArgs v) {
  extern __shared__ __align__(16) unsigned char smem[];
  recon2d_tile<T, NF, VelArgs, VK>(g, fp, gdisp, ord, stats, xcd_tile(blockIdx.x, ntiles),
                                   tiles_x, smem, nt, v);
}

}  // namespace sl
