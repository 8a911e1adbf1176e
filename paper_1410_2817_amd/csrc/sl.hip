// Forward semi-Lagrangian advection on gfx950: kernels and the C ABI of sl.h.
//
// One step of the scheme (Sec. 2 of Becerra-Sagredo, Malaga & Mandujano):
//   traj_kernel   one work-item per lattice node integrates its trajectory
//                 (RK4 or Williamson's low-storage RK3) and stores the FP64
//                 displacement in cell units, structure-of-arrays;
//   reconstruction, one work-item per mesh node: host-element walk + Newton
//                 on the multilinear element map (eq. "mapping1"), order
//                 selection from the jump flags of Sec. 2.3, cardinal
//                 Z-spline weights (Appendix) and the tensor-product
//                 gather-sum (eq. "multiZ").  2-D grids use the LDS-tiled
//                 kernel of sl_recon2d.h; 3-D grids compute the flags here
//                 (flags_kernel), reduce them to per-cell order words and run
//                 the kernel of sl_recon3d.h.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>
#include <tuple>
#include <utility>
#include <vector>

#include "sl.h"
#include "sl_device.h"
#include "sl_launch.h"
#include "sl_orders.h"
#include "sl_recon2d.h"
#include "sl_recon3d.h"
#include "sl_source.h"
#include "sl_traj.h"

namespace sl {

__global__ void zero_kernel(unsigned long long* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    p[i] = 0ull;
}

// Totals of the counter copies into the caller's array of sl_advance_static
// (one work-item per counter).
__global__ void static_counters_kernel(const unsigned long long* __restrict__ copies,
                                       int64_t* __restrict__ out) {
  const int slots[SL_STATIC_COUNTERS - 1] = {ST_SEARCH_FAIL, ST_NEWTON_FAIL, ST_NONFINITE,
                                             ST_ORDER0,      ST_ORDER1,      ST_WALKED,
                                             ST_SCANNED};
  const int k = threadIdx.x;
  if (k >= SL_STATIC_COUNTERS) return;
  unsigned long long sum = 0ull;
  if (k < SL_STATIC_COUNTERS - 1)
    for (int c = 0; c < kStatCopies; ++c) sum += copies[c * kStatStride + slots[k]];
  out[k] = (int64_t)sum;
}

}  // namespace sl

// Scratch of sl_advance_static: the workspace of callers that cannot
// allocate.  Each device holds its own copy; host code reaches it only
// through the address hipGetSymbolAddress returns on that device.
static __device__ __align__(256) unsigned char scratch[SL_STATIC_SCRATCH_BYTES];

// ===========================================================================
// Host side: descriptors, validation, launches.

#include "sl_grid.h"

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kStatsBytes = sizeof(unsigned long long) * sl::kStatWords;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

constexpr size_t kMaxPendingPairs = 8192;

void prof_fold(sl_grid* gr) {
  for (const sl_prof_pair& p : gr->pending) {
    float ms = 0.0f;
    if (hipEventSynchronize(p.stop) == hipSuccess &&
        hipEventElapsedTime(&ms, p.start, p.stop) == hipSuccess) {
      gr->prof_ms[p.kind] += ms;
      gr->prof_n[p.kind] += 1;
    }
    gr->ev_free.push_back(p.start);
    gr->ev_free.push_back(p.stop);
  }
  gr->pending.clear();
}

hipEvent_t prof_event(sl_grid* gr) {
  if (!gr->ev_free.empty()) {
    hipEvent_t e = gr->ev_free.back();
    gr->ev_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Events for the next launch of `kind` (null events when profiling is off).
struct ProfSlot {
  hipEvent_t start = nullptr, stop = nullptr;
};

// Every prof_period-th launch of each kind is timed (none when it is 0).
ProfSlot prof_begin(sl_grid* gr, int kind) {
  ProfSlot ps;
  if (gr->prof_period <= 0) return ps;
  if (gr->prof_count[kind]++ % gr->prof_period != 0) return ps;
  if (gr->pending.size() >= kMaxPendingPairs) prof_fold(gr);
  ps.start = prof_event(gr);
  ps.stop = prof_event(gr);
  if (!ps.start || !ps.stop) {
    if (ps.start) gr->ev_free.push_back(ps.start);
    if (ps.stop) gr->ev_free.push_back(ps.stop);
    ps.start = ps.stop = nullptr;
  }
  return ps;
}

void prof_end(sl_grid* gr, const ProfSlot& ps, int kind, hipError_t launched) {
  if (!ps.start) return;
  if (launched == hipSuccess) {
    gr->pending.push_back({kind, ps.start, ps.stop});
  } else {
    gr->ev_free.push_back(ps.start);
    gr->ev_free.push_back(ps.stop);
  }
}

// 2-D grids from this many nodes up take the separate order-word pass.
constexpr int64_t kWordsMinNodes = int64_t(1) << 22;

int check_desc(const sl_grid_desc* d) {
  if (!d) return SL_EINVAL;
  if (d->dim != 2 && d->dim != 3) return SL_EINVAL;
  if (d->nfields < 1 || d->nfields > SL_MAX_FIELDS) return SL_EINVAL;
  if (d->value_prec != SL_FP64 && d->value_prec != SL_FP32) return SL_EINVAL;
  if (d->order_max < 0 || d->order_max > 2) return SL_EINVAL;
  if (d->integrator != SL_RK4 && d->integrator != SL_RK3_WILLIAMSON) return SL_EINVAL;
  if (d->reconstruct_every < 1) return SL_EINVAL;
  if (d->newton_max_iter < 1 || d->newton_max_iter > 1000) return SL_EINVAL;
  if (!(d->newton_tol > 0.0) || !(d->eps_inside >= 0.0)) return SL_EINVAL;
  if (d->walk_max < 0 || d->walk_max > 4096) return SL_EINVAL;
  if (d->scan_radius < 0 || d->scan_radius > 16) return SL_EINVAL;
  if (d->limiter != 0 && d->limiter != 1) return SL_EINVAL;
  if (d->limiter_pass < SL_LIMITER_AUTO || d->limiter_pass > SL_LIMITER_ORDER_WORDS)
    return SL_EINVAL;
  if (d->limiter && !(d->limiter_theta >= 0.0)) return SL_EINVAL;
  int64_t tot = 1;
  for (int a = 0; a < d->dim; ++a) {
    // The quintic stencil must fit in the periodic grid once.
    if (d->n[a] < 6 || d->n[a] > (1 << 24)) return SL_EINVAL;
    if (!(d->length[a] > 0.0) || !isfinite(d->length[a])) return SL_EINVAL;
    tot *= d->n[a];
    if (tot > (int64_t)INT32_MAX / 2) return SL_EINVAL;
  }
  // Launch-grid limits of the y and z grid dimensions.
  if (d->n[1] > 4 * 65535 || (d->dim == 3 && d->n[2] > 65535)) return SL_EINVAL;
  const sl_velocity& v = d->vel;
  if (v.kind < SL_VEL_UNIFORM || v.kind > SL_VEL_CARRIED) return SL_EINVAL;
  if (v.kind == SL_VEL_CARRIED && d->nfields < d->dim) return SL_EINVAL;
  if (v.kind == SL_VEL_GRIDDED && !(v.p[0] == 0.0 || v.p[0] == 1.0 || v.p[0] == 2.0))
    return SL_EINVAL;
  if (v.kind == SL_VEL_SWIRL2D && (d->dim != 2 || !(v.p[0] != 0.0))) return SL_EINVAL;
  if (v.kind == SL_VEL_DEFORM3D && (d->dim != 3 || !(v.p[0] != 0.0))) return SL_EINVAL;
  if (v.kind == SL_VEL_FOURIER) {
    if (v.nmodes < 1 || v.nmodes > SL_MAX_MODES || !v.modes) return SL_EINVAL;
    for (int q = 0; q < v.nmodes; ++q) {
      double k2 = 0.0;
      for (int a = 0; a < d->dim; ++a) k2 += v.modes[7 * q + a] * v.modes[7 * q + a];
      if (!(k2 > 0.0)) return SL_EINVAL;
      for (int c = 0; c < 7; ++c)
        if (!isfinite(v.modes[7 * q + c])) return SL_EINVAL;
    }
  }
  for (int c = 0; c < 8; ++c)
    if (!isfinite(v.p[c])) return SL_EINVAL;
  bool shard = false;
  for (int a = 0; a < d->dim; ++a) {
    if (d->offset[a] <= -(int64_t(1) << 30) || d->offset[a] >= (int64_t(1) << 30))
      return SL_EINVAL;
    shard = shard || d->offset[a] != 0;
  }
  // Gridded samples and the source term's Coriolis parameter are indexed by
  // this grid's own nodes.
  if (shard && (v.kind == SL_VEL_GRIDDED || d->source != SL_SRC_NONE)) return SL_EINVAL;
  if (d->source != SL_SRC_NONE) {
    if (d->source != SL_SRC_SHALLOW_WATER) return SL_EINVAL;
    if (d->dim != 2 || v.kind != SL_VEL_CARRIED || d->nfields < 3) return SL_EINVAL;
    if (d->integrator != SL_RK3_WILLIAMSON || d->reconstruct_every != 1) return SL_EINVAL;
    for (int c = 0; c < 4; ++c)
      if (!isfinite(d->source_p[c])) return SL_EINVAL;
    if (d->source_p[3] < 0.0) return SL_EINVAL;
  }
  return SL_OK;
}

thread_local char g_detail[256] = "";

int hip_status(hipError_t e) {
  if (e == hipSuccess) return SL_OK;
  snprintf(g_detail, sizeof(g_detail), "%s: %s", hipGetErrorName(e), hipGetErrorString(e));
  return SL_EHIP;
}

// Launch errors are read back with hipGetLastError(); clear whatever another
// library left behind first so it is not reported as ours.
void clear_stale_error() { (void)hipGetLastError(); }

using sl::launch;

// Carried velocity: straight-line displacement from the fields `fp.in`.
template <int D>
hipError_t launch_carried(sl_grid* gr, const sl::FieldPtrs& fp, double* disp, double dt,
                          int accumulate, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const dim3 blocks((unsigned)((gr->g.n[0] + sl::kTrajBX - 1) / sl::kTrajBX),
                    (unsigned)((gr->g.n[1] + sl::kTrajBY - 1) / sl::kTrajBY),
                    (unsigned)gr->g.n[2]);
  const dim3 threads(sl::kTrajBX, sl::kTrajBY);
  if (gr->desc.value_prec == SL_FP32)
    return launch(sl::carried_traj_kernel<D, float>, blocks, threads, 0, s, e0, e1, gr->g, fp,
                  disp, dt, accumulate);
  return launch(sl::carried_traj_kernel<D, double>, blocks, threads, 0, s, e0, e1, gr->g, fp,
                disp, dt, accumulate);
}

// Time factors of the stages of a step over [t, t + dt].
sl::StageTimes stage_times(const sl_grid* gr, double t, double dt) {
  sl::StageTimes st;
  const bool periodic = gr->v.kind == SL_VEL_SWIRL2D || gr->v.kind == SL_VEL_DEFORM3D;
  const double ts[4] = {t, gr->desc.integrator == SL_RK4 ? t + 0.5 * dt : t + dt / 3.0,
                        gr->desc.integrator == SL_RK4 ? t + dt : t + 0.75 * dt, t + dt};
  for (int i = 0; i < 4; ++i) st.tf[i] = periodic ? cos(M_PI * ts[i] / gr->v.p[0]) : 1.0;
  return st;
}

// `trig`: the grid's table (fresh lattice), or null.
template <int D>
hipError_t launch_traj(sl_grid* gr, double* disp, double t, double dt, int accumulate,
                       hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                       const double* trig = nullptr) {
  const sl::StageTimes st = stage_times(gr, t, dt);
  const dim3 blocks((unsigned)((gr->g.n[0] + sl::kTrajBX - 1) / sl::kTrajBX),
                    (unsigned)((gr->g.n[1] + sl::kTrajBY - 1) / sl::kTrajBY),
                    (unsigned)gr->g.n[2]);
  const dim3 threads(sl::kTrajBX, sl::kTrajBY);
  const int integ = gr->desc.integrator;
  switch (gr->v.kind) {
    case SL_VEL_UNIFORM:
      return launch(sl::traj_kernel<D, SL_VEL_UNIFORM>, blocks, threads, 0, s, e0, e1, gr->g, gr->v, disp, st, dt, accumulate, integ, trig);
    case SL_VEL_SOLID_BODY:
      return launch(sl::traj_kernel<D, SL_VEL_SOLID_BODY>, blocks, threads, 0, s, e0, e1, gr->g, gr->v, disp, st, dt, accumulate, integ, trig);
    case SL_VEL_SWIRL2D:
      return launch(sl::traj_kernel<D, SL_VEL_SWIRL2D>, blocks, threads, 0, s, e0, e1, gr->g, gr->v, disp, st, dt, accumulate, integ, trig);
    case SL_VEL_DEFORM3D:
      return launch(sl::traj_kernel<D, SL_VEL_DEFORM3D>, blocks, threads, 0, s, e0, e1, gr->g, gr->v, disp, st, dt, accumulate, integ, trig);
    case SL_VEL_GRIDDED:
      if constexpr (D == 2) {
        // Tiles with their velocity samples staged in LDS.
        const int tx = (gr->g.n[0] + sl::kGridTile - 1) / sl::kGridTile;
        const int ty = (gr->g.n[1] + sl::kGridTile - 1) / sl::kGridTile;
        return launch(sl::traj_gridded2d_kernel<2>, dim3(tx * ty), dim3(256), 0, s, e0, e1, gr->g,
                      gr->v, disp, st, dt, accumulate, integ, tx);
      }
      return launch(sl::traj_kernel<D, SL_VEL_GRIDDED>, blocks, threads, 0, s, e0, e1, gr->g, gr->v, disp, st, dt, accumulate, integ, trig);
    default:
      return launch(sl::traj_kernel<D, SL_VEL_FOURIER>, blocks, threads, 0, s, e0, e1, gr->g, gr->v, disp, st, dt, accumulate, integ, trig);
  }
}

// Limiter order words of the fields `fp.in` (none when the limiter is off):
// flag bytes, then one window pass per axis.  *ord receives the word array
// (in the workspace); e0 / e1 are recorded by the first / last launch.
template <int D, typename T>
hipError_t launch_order_words(sl_grid* gr, const sl::FieldPtrs& fp, char* ws, hipStream_t s,
                              hipEvent_t e0, hipEvent_t e1, const uint16_t** ord) {
  *ord = nullptr;
  if (!(gr->g.limiter && gr->g.order_max > 0) || !gr->limiter_words) return hipSuccess;
  uint8_t* flags = reinterpret_cast<uint8_t*>(ws + gr->off_flags);
  uint16_t* wa = reinterpret_cast<uint16_t*>(ws + gr->off_ord);
  uint16_t* wb = wa + gr->ntot;
  const dim3 wt(64, 4);
  // Quad kernels when rows are a multiple of 4 nodes and the fields are
  // 16-byte aligned.
  bool quad = gr->g.n[0] % 4 == 0;
  for (int f = 0; f < gr->g.nfields; ++f) quad = quad && ((uintptr_t)fp.in[f] % 16) == 0;
  hipError_t e;
  if (quad) {
    const dim3 qb((unsigned)((gr->g.n[0] / 4 + 63) / 64), (unsigned)((gr->g.n[1] + 3) / 4),
                  (unsigned)gr->g.n[2]);
    auto* qa = reinterpret_cast<unsigned long long*>(wa);
    auto* qb2 = reinterpret_cast<unsigned long long*>(wb);
    const int nq = gr->g.n[0] / 4;
    if (nq <= sl::kBlock) {
      // Whole rows per workgroup: flags and x window in one pass.
      const int rows = sl::kBlock / nq;
      const dim3 fb((unsigned)((gr->g.n[1] + rows - 1) / rows), (unsigned)gr->g.n[2]);
      e = launch(sl::flags_window_x_kernel<D, T>, fb, dim3(sl::kBlock), 0, s, e0, nullptr,
                 gr->g, fp, qa);
    } else {
      auto* f4 = reinterpret_cast<uint32_t*>(flags);
      e = launch(sl::flags_quad_kernel<D, T>, qb, wt, 0, s, e0, nullptr, gr->g, fp, f4);
      if (e == hipSuccess)
        e = launch(sl::window_x_quad_kernel, qb, wt, 0, s, nullptr, nullptr, gr->g,
                   (const uint32_t*)f4, qa);
    }
    if (e == hipSuccess && D == 2)
      e = launch(sl::window_yz_quad_kernel<1>, qb, wt, 0, s, nullptr, e1, gr->g,
                 (const unsigned long long*)qa, qb2);
    if (e == hipSuccess && D == 3) {
      // The y and z windows in one pass, marching through chunks of planes.
      const dim3 zb(qb.x, qb.y, (unsigned)((gr->g.n[2] + sl::kZChunk - 1) / sl::kZChunk));
      e = launch(sl::window_yz3_quad_kernel, zb, wt, 0, s, nullptr, e1, gr->g,
                 (const unsigned long long*)qa, qb2);
    }
    *ord = wb;
    return e;
  } else {
    const dim3 fb((unsigned)((gr->ntot + sl::kBlock - 1) / sl::kBlock)), ft(sl::kBlock);
    e = launch(sl::flags_kernel<D, T>, fb, ft, 0, s, e0, nullptr, gr->g, fp, flags);
    const dim3 wbk((unsigned)((gr->g.n[0] + 63) / 64), (unsigned)((gr->g.n[1] + 3) / 4),
                   (unsigned)gr->g.n[2]);
    if (e == hipSuccess)
      e = launch(sl::window_or_kernel<0>, wbk, wt, 0, s, nullptr, nullptr, gr->g,
                 (const uint8_t*)flags, (const uint16_t*)nullptr, wa);
    if (e == hipSuccess)
      e = launch(sl::window_or_kernel<1>, wbk, wt, 0, s, nullptr, D == 2 ? e1 : nullptr, gr->g,
                 (const uint8_t*)nullptr, (const uint16_t*)wa, wb);
    if (e == hipSuccess && D == 3)
      e = launch(sl::window_or_kernel<2>, wbk, wt, 0, s, nullptr, e1, gr->g,
                 (const uint8_t*)nullptr, (const uint16_t*)wb, wa);
  }
  *ord = D == 3 ? wa : wb;
  return e;
}

template <int D, typename T>
hipError_t launch_recon(sl_grid* gr, const sl::FieldPtrs& fp, char* ws, const double* disp,
                        const uint16_t* ord, const sl::NextTraj& nt, hipStream_t s,
                        hipEvent_t e0, hipEvent_t e1) {
  auto* stats = reinterpret_cast<unsigned long long*>(ws + gr->off_stats);
  if constexpr (D == 2) {
    // Tile shape does not depend on the field count.
    using C = sl::Tile2D<T, 1>;
    const int tiles_x = (gr->g.n[0] + C::TX - 1) / C::TX;
    const int tiles_y = (gr->g.n[1] + C::TY - 1) / C::TY;
    const int ntiles = tiles_x * tiles_y;
    const dim3 grid(ntiles), block(sl::kTileThreads);
#define SL_RECON2D(NF)                                                                    \
  case NF:                                                                                \
    return launch(sl::recon2d_tiled_kernel<T, NF>, grid, block,                          \
                  (uint32_t)sl::Tile2D<T, NF>::LDS_BYTES, s, e0, e1, gr->g, fp, disp, \
                  ord, stats, tiles_x, ntiles, nt, gr->v);
    // The swirl with three fields has a kernel of its own, whose fused
    // trajectories are that family's alone (10 scalar registers spilled
    // against 16): 1024^2 step 45.2 -> 44.4 us, 4096^2 0.599 -> 0.589 ms.
    // A carried velocity with three FP64 fields (the shallow-water system)
    // runs a kernel without the fused trajectories, at five waves per SIMD.
    if constexpr (sizeof(T) == 8) {
      if (gr->g.nfields == 3 && gr->v.kind == SL_VEL_CARRIED)
        return launch(sl::recon2d_tiled_kernel<T, 3, SL_VEL_CARRIED>, grid, block,
                      (uint32_t)sl::Tile2D<T, 3>::LDS_BYTES, s, e0, e1, gr->g, fp, disp, ord,
                      stats, tiles_x, ntiles, nt, gr->v);
    }
    if (gr->g.nfields == 3 && gr->v.kind == SL_VEL_SWIRL2D)
      return launch(sl::recon2d_tiled_kernel<T, 3, SL_VEL_SWIRL2D>, grid, block,
                    (uint32_t)sl::Tile2D<T, 3>::LDS_BYTES, s, e0, e1, gr->g, fp, disp, ord, stats,
                    tiles_x, ntiles, nt, gr->v);
    switch (gr->g.nfields) {
      SL_RECON2D(1)
      SL_RECON2D(2)
      SL_RECON2D(3)
      SL_RECON2D(4)
      SL_RECON2D(5)
      SL_RECON2D(6)
      SL_RECON2D(7)
      default:
        return launch(sl::recon2d_tiled_kernel<T, 8>, grid, block,
                      (uint32_t)sl::Tile2D<T, 8>::LDS_BYTES, s, e0, e1, gr->g, fp, disp,
                      ord, stats, tiles_x, ntiles, nt, gr->v);
    }
#undef SL_RECON2D
  } else {
    using C = sl::Tile3D;
    const int tiles_x = (gr->g.n[0] + C::TX - 1) / C::TX;
    const int tiles_y = (gr->g.n[1] + C::TY - 1) / C::TY;
    const int tiles_z = (gr->g.n[2] + C::TZ - 1) / C::TZ;
    const int ntiles = tiles_x * tiles_y * tiles_z;
    // Buffer offsets are signed 32-bit byte offsets within one field.
    const int buf_ok = (size_t)gr->ntot * sizeof(T) <= (size_t)INT32_MAX;
    const int dbuf_ok = (size_t)gr->ntot * sizeof(double) <= (size_t)INT32_MAX;
    const dim3 grid(ntiles), block(sl::kTileThreads);
#define SL_RECON3D(NF)                                                                       \
  case NF:                                                                                   \
    return launch(sl::recon3d_kernel<T, NF>, grid, block, 0, s, e0, e1, gr->g, fp, disp, ord, \
                  stats, tiles_x, tiles_y, ntiles, buf_ok, dbuf_ok, nt, gr->v);
    // The deformational flow with one field (the paper's 3-D test) has a
    // kernel of its own: 0.6 % (FP64) to 1 % (FP32 values) faster per step.
    // So do Fourier flows with three fields, whose registers then cover that
    // family's trajectories alone (4 VGPRs and 11 scalar registers spilled
    // against 5 and 12): 256^3 step 1.82 -> 1.80 ms.
    if (gr->g.nfields == 1 && gr->v.kind == SL_VEL_DEFORM3D)
      return launch(sl::recon3d_kernel<T, 1, SL_VEL_DEFORM3D>, grid, block, 0, s, e0, e1, gr->g,
                    fp, disp, ord, stats, tiles_x, tiles_y, ntiles, buf_ok, dbuf_ok, nt, gr->v);
    if (gr->g.nfields == 3 && gr->v.kind == SL_VEL_FOURIER)
      return launch(sl::recon3d_kernel<T, 3, SL_VEL_FOURIER>, grid, block, 0, s, e0, e1, gr->g,
                    fp, disp, ord, stats, tiles_x, tiles_y, ntiles, buf_ok, dbuf_ok, nt, gr->v);
    switch (gr->g.nfields) {
      SL_RECON3D(1)
      SL_RECON3D(2)
      SL_RECON3D(3)
      SL_RECON3D(4)
      SL_RECON3D(5)
      SL_RECON3D(6)
      SL_RECON3D(7)
      default:
        return launch(sl::recon3d_kernel<T, 8>, grid, block, 0, s, e0, e1, gr->g, fp, disp, ord,
                      stats, tiles_x, tiles_y, ntiles, buf_ok, dbuf_ok, nt, gr->v);
    }
#undef SL_RECON3D
  }
}

}  // namespace

extern "C" {

void sl_grid_desc_init(sl_grid_desc* d) {
  if (!d) return;
  memset(d, 0, sizeof(*d));
  d->dim = 2;
  d->n[0] = d->n[1] = d->n[2] = 64;
  d->length[0] = d->length[1] = d->length[2] = 1.0;
  d->nfields = 1;
  d->value_prec = SL_FP64;
  d->order_max = 2;
  d->limiter = 0;
  d->limiter_theta = 0.25;
  d->integrator = SL_RK4;
  d->reconstruct_every = 1;
  d->vel.kind = SL_VEL_UNIFORM;
  d->newton_max_iter = 20;
  d->newton_tol = 1e-14;
  d->walk_max = 32;
  d->scan_radius = 4;
  d->eps_inside = 1e-12;
}

int sl_create_grid(const sl_grid_desc* desc, sl_grid** out) {
  if (!out) return SL_EINVAL;
  *out = nullptr;
  const int rc = check_desc(desc);
  if (rc != SL_OK) return rc;
  sl_grid* gr = new (std::nothrow) sl_grid();
  if (!gr) return SL_ENOMEM;
  gr->desc = *desc;
  const int D = desc->dim;
  if (desc->vel.kind == SL_VEL_FOURIER) {
    gr->modes.assign(desc->vel.modes, desc->vel.modes + 7 * desc->vel.nmodes);
    gr->desc.vel.modes = gr->modes.data();
  } else {
    gr->desc.vel.modes = nullptr;
    gr->desc.vel.nmodes = 0;
  }
  sl::GridArgs& g = gr->g;
  memset(&g, 0, sizeof(g));
  gr->ntot = 1;
  for (int a = 0; a < 3; ++a) {
    g.n[a] = a < D ? (int)desc->n[a] : 1;
    g.h[a] = a < D ? desc->length[a] / (double)desc->n[a] : 1.0;
    g.rh[a] = 1.0 / g.h[a];
    g.r6h[a] = 1.0 / (6.0 * g.h[a]);
    g.off[a] = a < D ? (int)desc->offset[a] : 0;
    if (a < D) gr->ntot *= desc->n[a];
  }
  g.ntot = (int)gr->ntot;
  g.nfields = desc->nfields;
  g.order_max = desc->order_max;
  g.limiter = desc->limiter;
  g.theta = desc->limiter_theta;
  g.newton_max_iter = desc->newton_max_iter;
  g.newton_tol = desc->newton_tol;
  g.walk_max = desc->walk_max;
  g.scan_radius = desc->scan_radius;
  g.eps = desc->eps_inside;

  sl::VelArgs& v = gr->v;
  memset(&v, 0, sizeof(v));
  v.kind = desc->vel.kind;
  for (int c = 0; c < 8; ++c) v.p[c] = desc->vel.p[c];
  if (v.kind == SL_VEL_GRIDDED) {
    v.ug_m = (int)desc->vel.p[0];
    for (int a = 0; a < 3; ++a) {
      v.ug_n[a] = g.n[a];
      v.ug_h[a] = g.h[a];
    }
  }
  if (v.kind == SL_VEL_FOURIER) {
    v.nmodes = desc->vel.nmodes;
    const double pi = M_PI;
    // 2-D integer wave vectors with small components take the encoding whose
    // modes share e^{i pi y_a} (sl::Mode).  In 3-D the three product loops per
    // mode measured no faster than the cosine per mode, and slower inside the
    // fused reconstruction (fewer waves in flight to hide their scalar loads).
    v.small_k = D == 2;
    for (int q = 0; q < v.nmodes; ++q)
      for (int a = 0; a < D; ++a) {
        const double k = gr->modes[7 * q + a];
        v.small_k = v.small_k && k == std::nearbyint(k) && std::fabs(k) <= sl::kSmallK;
      }
    for (int a = 0; a < D; ++a) v.kscale[a] = 2.0 / desc->length[a];
    for (int q = 0; q < v.nmodes; ++q) {
      const double* md = gr->modes.data() + 7 * q;
      double k2 = 0.0, kp[3] = {0.0, 0.0, 0.0};
      for (int a = 0; a < D; ++a) {
        k2 += md[a] * md[a];
        kp[a] = md[a] / desc->length[a];
      }
      if (v.small_k) {
        v.mode[q].ik.cphi = std::cos(md[6]);
        v.mode[q].ik.sphi = std::sin(md[6]);
        for (int a = 0; a < D; ++a) v.mode[q].ik.k[a] = (int)md[a];
      } else {
        for (int a = 0; a < D; ++a) v.mode[q].gen.c[a] = 2.0 * kp[a];
        v.mode[q].gen.phase_over_pi = md[6] / pi;
      }
      const double s = desc->vel.p[0] * 2.0 * pi / k2;
      if (D == 2) {
        v.mode[q].amp[0] = s * md[3] * kp[1];
        v.mode[q].amp[1] = -s * md[3] * kp[0];
      } else {
        // curl(a sin(theta)) = cos(theta) grad(theta) x a
        v.mode[q].amp[0] = s * (kp[1] * md[5] - kp[2] * md[4]);
        v.mode[q].amp[1] = s * (kp[2] * md[3] - kp[0] * md[5]);
        v.mode[q].amp[2] = s * (kp[0] * md[4] - kp[1] * md[3]);
      }
    }
  }
  // Bound on the Runge-Kutta stage offsets per unit dt in the argument of the
  // angle-shift evaluators: max |u_a| (times y_a / x_a for the Fourier ik
  // encoding) times the integrator's factor.  RK4 evaluates at most dt u
  // away; Williamson's RK3 at most dt max|u| (1/3 + 15/16 * 14/9) < 1.8.
  {
    double umax = HUGE_VAL;
    if (v.kind == SL_VEL_SWIRL2D) {
      umax = std::fabs(v.p[1]);  // |sin^2(pi x) sin(2 pi y)| <= 1
    } else if (v.kind == SL_VEL_DEFORM3D) {
      umax = 2.0 * std::fabs(v.p[1]);  // u_x carries the factor 2
    } else if (v.kind == SL_VEL_FOURIER && v.small_k) {
      umax = 0.0;
      for (int a = 0; a < D; ++a) {
        double sa = 0.0;
        for (int q = 0; q < v.nmodes; ++q) sa += std::fabs(v.mode[q].amp[a]);
        umax = std::max(umax, sa * v.kscale[a]);
      }
    }
    v.shift_rate = umax * (desc->integrator == SL_RK4 ? 1.0 : 1.8);
  }
  gr->off_stats = 0;
  gr->off_disp = align_up(kStatsBytes);
  gr->off_flags = align_up(gr->off_disp + sizeof(double) * (size_t)D * (size_t)gr->ntot);
  // Two 16-bit limiter window words per node (ping-pong).
  gr->off_ord = align_up(gr->off_flags + (size_t)gr->ntot);
  // Second displacement buffer: sl_advance integrates the next step's
  // trajectories there while the current step reconstructs.
  gr->off_disp2 = align_up(gr->off_ord + 4 * (size_t)gr->ntot);
  gr->ws_bytes = align_up(gr->off_disp2 + sizeof(double) * (size_t)D * (size_t)gr->ntot);
  if (desc->source != SL_SRC_NONE) {
    const size_t vbytes = (desc->value_prec == SL_FP32 ? 4 : 8) * (size_t)gr->ntot;
    const size_t plane = sizeof(double) * (size_t)gr->ntot;
    gr->off_src_h = gr->ws_bytes;
    gr->off_src_g = align_up(gr->off_src_h + (size_t)desc->nfields * vbytes);
    gr->off_src_qx = align_up(gr->off_src_g + (size_t)desc->nfields * vbytes);
    gr->off_src_qh = align_up(gr->off_src_qx + 2 * plane);
    gr->ws_bytes = align_up(gr->off_src_qh + 3 * plane);
  }
  gr->off_trig = gr->trig_bytes = 0;
  if (sl::uses_trig_table(v, D) && desc->source == SL_SRC_NONE) {
    gr->off_trig = gr->ws_bytes;
    gr->trig_bytes = 2 * sizeof(double) * sl::trig_table_pairs(g, D);
    gr->ws_bytes = align_up(gr->off_trig + gr->trig_bytes);
  }
  // 2-D grids evaluate the limiter flags inside the reconstruction tiles
  // (the values are staged there anyway) unless the grid is large, where a
  // separate order-word pass costs less than the tiles' redundant flag work;
  // the descriptor may force either choice.
  gr->limiter_words = D == 3 || desc->limiter_pass == SL_LIMITER_ORDER_WORDS ||
                      (desc->limiter_pass == SL_LIMITER_AUTO && gr->ntot >= kWordsMinNodes);
  gr->steps_since_reset = 0;
  *out = gr;
  return SL_OK;
}

int sl_destroy_grid(sl_grid* grid) {
  if (!grid) return SL_OK;
  for (const sl_prof_pair& p : grid->pending) {
    (void)hipEventSynchronize(p.stop);
    grid->ev_free.push_back(p.start);
    grid->ev_free.push_back(p.stop);
  }
  for (hipEvent_t e : grid->ev_free) (void)hipEventDestroy(e);
  delete grid;
  return SL_OK;
}

size_t sl_workspace_bytes(const sl_grid* grid) { return grid ? grid->ws_bytes : 0; }

int sl_set_velocity_field(sl_grid* gr, const double* const* components) {
  if (!gr || !components || gr->v.kind != SL_VEL_GRIDDED) return SL_EINVAL;
  for (int a = 0; a < gr->desc.dim; ++a)
    if (!components[a]) return SL_EINVAL;
  for (int a = 0; a < gr->desc.dim; ++a) gr->v.ug[a] = components[a];
  return SL_OK;
}

int sl_step(sl_grid* gr, void* workspace, double t, double dt, void* stream) {
  if (!gr || !workspace || !isfinite(t) || !isfinite(dt)) return SL_EINVAL;
  if (gr->v.kind == SL_VEL_CARRIED) return SL_EINVAL;  // needs the fields: sl_advance
  if (gr->v.kind == SL_VEL_GRIDDED && !gr->v.ug[0]) return SL_ESTATE;
  if (((uintptr_t)workspace) % kAlign) return SL_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  double* disp = reinterpret_cast<double*>(static_cast<char*>(workspace) + gr->off_disp);
  const int acc = gr->steps_since_reset > 0;
  clear_stale_error();
  const ProfSlot ps = prof_begin(gr, 0);
  const hipError_t e = gr->desc.dim == 2
                           ? launch_traj<2>(gr, disp, t, dt, acc, s, ps.start, ps.stop)
                           : launch_traj<3>(gr, disp, t, dt, acc, s, ps.start, ps.stop);
  prof_end(gr, ps, 0, e);
  const int rc = hip_status(e);
  if (rc == SL_OK) {
    gr->steps_since_reset++;
    gr->steps_launched++;
  }
  return rc;
}

}  // extern "C"

namespace {

// Field pointer block for in -> out after the checks of sl_reconstruct.
int field_ptrs(const sl_grid* gr, const void* const* in, void* const* out, sl::FieldPtrs* fp) {
  if (!in || !out) return SL_EINVAL;
  memset(fp, 0, sizeof(*fp));
  const int nf = gr->desc.nfields;
  for (int f = 0; f < nf; ++f) {
    if (!in[f] || !out[f]) return SL_EINVAL;
    fp->in[f] = in[f];
    fp->out[f] = out[f];
  }
  for (int f = 0; f < nf; ++f)
    for (int q = 0; q < nf; ++q)
      if (fp->out[f] == fp->in[q]) return SL_EINVAL;
  return SL_OK;
}

// Order words (if any) and the reconstruction from displacement `disp`; the
// reconstruction kernel also integrates the trajectories `nt` asks for.
hipError_t reconstruct_launches(sl_grid* gr, char* ws, const sl::FieldPtrs& fp,
                                const double* disp, const sl::NextTraj& nt, hipStream_t s) {
  const bool f32 = gr->desc.value_prec == SL_FP32;
  const ProfSlot po = prof_begin(gr, 2);
  const uint16_t* ord = nullptr;
  hipError_t e;
  if (gr->desc.dim == 2)
    e = f32 ? launch_order_words<2, float>(gr, fp, ws, s, po.start, po.stop, &ord)
            : launch_order_words<2, double>(gr, fp, ws, s, po.start, po.stop, &ord);
  else
    e = f32 ? launch_order_words<3, float>(gr, fp, ws, s, po.start, po.stop, &ord)
            : launch_order_words<3, double>(gr, fp, ws, s, po.start, po.stop, &ord);
  prof_end(gr, po, 2, ord ? e : hipErrorInvalidValue);  // no launch: drop the pair
  if (e != hipSuccess) return e;
  const ProfSlot ps = prof_begin(gr, 1);
  if (gr->desc.dim == 2)
    e = f32 ? launch_recon<2, float>(gr, fp, ws, disp, ord, nt, s, ps.start, ps.stop)
            : launch_recon<2, double>(gr, fp, ws, disp, ord, nt, s, ps.start, ps.stop);
  else
    e = f32 ? launch_recon<3, float>(gr, fp, ws, disp, ord, nt, s, ps.start, ps.stop)
            : launch_recon<3, double>(gr, fp, ws, disp, ord, nt, s, ps.start, ps.stop);
  prof_end(gr, ps, 1, e);
  return e;
}

// sl_advance with a source term (SL_SRC_SHALLOW_WATER): per step three
// Runge-Kutta stages of the lattice (one fused right-hand-side + stage kernel
// each), the stage fields between them reconstructed on the mesh, and the
// final reconstruction into the other field set.
template <typename T, int M>
hipError_t advance_source(sl_grid* gr, char* ws, void* const* fields_a, void* const* fields_b,
                          double dt, int nsteps, hipStream_t s) {
  // Williamson's 2N-storage third-order scheme.
  static const double kA[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
  static const double kB[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};
  const int nf = gr->desc.nfields;
  const size_t vbytes = sizeof(T) * (size_t)gr->ntot;
  double* disp = reinterpret_cast<double*>(ws + gr->off_disp);
  double* qx = reinterpret_cast<double*>(ws + gr->off_src_qx);
  double* qh = reinterpret_cast<double*>(ws + gr->off_src_qh);
  T* H[SL_MAX_FIELDS];
  T* G[SL_MAX_FIELDS];
  for (int f = 0; f < nf; ++f) {
    H[f] = reinterpret_cast<T*>(ws + gr->off_src_h + (size_t)f * vbytes);
    G[f] = reinterpret_cast<T*>(ws + gr->off_src_g + (size_t)f * vbytes);
  }
  sl::FieldPtrs to_stage, to_next;  // lattice values -> stage fields / result
  memset(&to_stage, 0, sizeof(to_stage));
  for (int f = 0; f < nf; ++f) {
    to_stage.in[f] = H[f];
    to_stage.out[f] = G[f];
  }
  const sl::SrcArgs sa{gr->desc.source_p[0], gr->desc.source_p[1], gr->desc.source_p[2],
                       gr->desc.source_p[3]};
  constexpr int TT = sl::StageTile::T;
  const int tiles_x = (gr->g.n[0] + TT - 1) / TT, tiles_y = (gr->g.n[1] + TT - 1) / TT;
  const int ntiles = tiles_x * tiles_y;
  hipError_t e = hipSuccess;
  for (int k = 0; k < nsteps && e == hipSuccess; ++k) {
    void* const* cur = (k & 1) ? fields_b : fields_a;
    void* const* nxt = (k & 1) ? fields_a : fields_b;
    gr->steps_launched++;
    for (int st = 0; st < 3 && e == hipSuccess; ++st) {
      if (st > 0) {
        e = reconstruct_launches(gr, ws, to_stage, disp, sl::NextTraj{}, s);
        if (e != hipSuccess) break;
        gr->reconstructs_launched++;
      }
      const T* gs[3];
      for (int c = 0; c < 3; ++c)
        gs[c] = st == 0 ? static_cast<const T*>(cur[c]) : static_cast<const T*>(G[c]);
      sl::FieldPtrs fp;
      memset(&fp, 0, sizeof(fp));
      for (int f = 0; f < nf; ++f) {
        fp.in[f] = cur[f];
        fp.out[f] = H[f];
      }
      const sl::SrcStage ss{kA[st], kB[st], dt, st == 0 ? 1 : 0, st == 2 ? 1 : 0};
      const ProfSlot p1 = prof_begin(gr, 3);
      e = launch(sl::sw_stage_kernel<T, M>, dim3(ntiles), dim3(256), 0, s, p1.start, p1.stop,
                 gr->g, sa, ss, fp, gs[0], gs[1], gs[2], disp, qx, qh, tiles_x, ntiles);
      prof_end(gr, p1, 3, e);
    }
    if (e != hipSuccess) break;
    memset(&to_next, 0, sizeof(to_next));
    for (int f = 0; f < nf; ++f) {
      to_next.in[f] = H[f];
      to_next.out[f] = nxt[f];
    }
    e = reconstruct_launches(gr, ws, to_next, disp, sl::NextTraj{}, s);
    if (e == hipSuccess) gr->reconstructs_launched++;
  }
  return e;
}

}  // namespace

extern "C" {

int sl_reconstruct(sl_grid* gr, void* workspace, const void* const* fields_in,
                   void* const* fields_out, void* stream) {
  if (!gr || !workspace || !fields_in || !fields_out) return SL_EINVAL;
  if (((uintptr_t)workspace) % kAlign) return SL_EINVAL;
  if (gr->steps_since_reset < 1) return SL_ESTATE;
  sl::FieldPtrs fp;
  const int prc = field_ptrs(gr, fields_in, fields_out, &fp);
  if (prc != SL_OK) return prc;
  char* ws = static_cast<char*>(workspace);
  clear_stale_error();
  const hipError_t e = reconstruct_launches(gr, ws, fp,
                                            reinterpret_cast<const double*>(ws + gr->off_disp),
                                            sl::NextTraj{}, static_cast<hipStream_t>(stream));
  const int rc = hip_status(e);
  if (rc == SL_OK) {
    gr->steps_since_reset = 0;
    gr->reconstructs_launched++;
  }
  return rc;
}

int sl_sync(sl_grid* gr, void* workspace, void* stream, sl_stats* out) {
  if (!gr || !workspace) return SL_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned long long copies[sl::kStatWords], host[sl::ST_COUNT];
  auto* dev = reinterpret_cast<unsigned long long*>(static_cast<char*>(workspace) + gr->off_stats);
  clear_stale_error();
  int rc = hip_status(hipMemcpyAsync(copies, dev, sizeof(copies), hipMemcpyDeviceToHost, s));
  if (rc != SL_OK) return rc;
  sl::zero_kernel<<<4, 256, 0, s>>>(dev, sl::kStatWords);
  rc = hip_status(hipGetLastError());
  if (rc != SL_OK) return rc;
  rc = hip_status(hipStreamSynchronize(s));
  if (rc != SL_OK) return rc;
  sl::stat_totals(copies, host);
  const int64_t recs = gr->reconstructs_launched;
  const int64_t nodes = recs * gr->ntot;
  if (out) {
    memset(out, 0, sizeof(*out));
    out->nodes = nodes;
    out->search_fail = (int64_t)host[sl::ST_SEARCH_FAIL];
    out->newton_fail = (int64_t)host[sl::ST_NEWTON_FAIL];
    out->nonfinite = (int64_t)host[sl::ST_NONFINITE];
    out->order_hist[0] = (int64_t)host[sl::ST_ORDER0];
    out->order_hist[1] = (int64_t)host[sl::ST_ORDER1];
    out->order_hist[2] = (int64_t)host[sl::ST_ORDER2];
    out->walked = (int64_t)host[sl::ST_WALKED];
    out->scanned = (int64_t)host[sl::ST_SCANNED];
    out->steps = gr->steps_launched;
    out->reconstructs = recs;
  }
  gr->steps_launched = 0;
  gr->reconstructs_launched = 0;
  if (host[sl::ST_SEARCH_FAIL]) return SL_ESEARCH;
  if (host[sl::ST_NEWTON_FAIL]) return SL_ENEWTON;
  if (host[sl::ST_NONFINITE]) return SL_ENONFINITE;
  return SL_OK;
}

int sl_advance(sl_grid* gr, void* workspace, void* const* fields_a, void* const* fields_b,
               double t0, double dt, int nsteps, void* stream, int* result_in_b) {
  if (!gr || !workspace || !fields_a || !fields_b || nsteps < 0) return SL_EINVAL;
  const int K = gr->desc.reconstruct_every;
  if (nsteps % K) return SL_EINVAL;
  if (gr->steps_since_reset != 0) return SL_ESTATE;
  if (gr->v.kind == SL_VEL_GRIDDED && !gr->v.ug[0]) return SL_ESTATE;
  if (gr->desc.source != SL_SRC_NONE) {
    if (((uintptr_t)workspace) % kAlign) return SL_EINVAL;
    sl::FieldPtrs ab, ba;
    int rc = field_ptrs(gr, (const void* const*)fields_a, fields_b, &ab);
    if (rc == SL_OK) rc = field_ptrs(gr, (const void* const*)fields_b, fields_a, &ba);
    if (rc != SL_OK) return rc;
    if (!isfinite(dt)) return SL_EINVAL;
    char* ws = static_cast<char*>(workspace);
    hipStream_t s = static_cast<hipStream_t>(stream);
    clear_stale_error();
    const bool f32 = gr->desc.value_prec == SL_FP32;
    const bool m1 = gr->desc.order_max < 2;  // three-point rules below Z2
    hipError_t e;
    if (f32)
      e = m1 ? advance_source<float, 1>(gr, ws, fields_a, fields_b, dt, nsteps, s)
             : advance_source<float, 2>(gr, ws, fields_a, fields_b, dt, nsteps, s);
    else
      e = m1 ? advance_source<double, 1>(gr, ws, fields_a, fields_b, dt, nsteps, s)
             : advance_source<double, 2>(gr, ws, fields_a, fields_b, dt, nsteps, s);
    if (e == hipSuccess && result_in_b) *result_in_b = nsteps & 1;
    return hip_status(e);
  }
  if (K == 1 && nsteps > 0 && gr->v.kind != SL_VEL_GRIDDED) {
    // Each reconstruction also integrates the next step's trajectories into
    // the other displacement buffer, so a step is one reconstruction launch
    // (plus the limiter order words) after the first step's trajectories.
    if (!workspace || ((uintptr_t)workspace) % kAlign) return SL_EINVAL;
    sl::FieldPtrs ab, ba;
    int rc = field_ptrs(gr, (const void* const*)fields_a, fields_b, &ab);
    if (rc == SL_OK) rc = field_ptrs(gr, (const void* const*)fields_b, fields_a, &ba);
    if (rc != SL_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* ws = static_cast<char*>(workspace);
    double* dbuf[2] = {reinterpret_cast<double*>(ws + gr->off_disp),
                       reinterpret_cast<double*>(ws + gr->off_disp2)};
    clear_stale_error();
    const bool carried = gr->v.kind == SL_VEL_CARRIED;
    hipError_t e = hipSuccess;
    // Every step's trajectories start from sin/cos(pi x) at the mesh nodes:
    // one table per call, n_x + n_y (+ n_z) entries (sl::trig_table_kernel).
    const double* trig = nullptr;
    if (gr->trig_bytes && !carried) {
      double* tb = reinterpret_cast<double*>(ws + gr->off_trig);
      e = gr->desc.dim == 2 ? sl::launch_trig_table<2>(gr->g, gr->v, tb, s)
                            : sl::launch_trig_table<3>(gr->g, gr->v, tb, s);
      trig = tb;
    }
    const ProfSlot ps = prof_begin(gr, 0);
    if (e == hipSuccess && carried)
      e = gr->desc.dim == 2 ? launch_carried<2>(gr, ab, dbuf[0], dt, 0, s, ps.start, ps.stop)
                            : launch_carried<3>(gr, ab, dbuf[0], dt, 0, s, ps.start, ps.stop);
    else if (e == hipSuccess)
      e = gr->desc.dim == 2
              ? launch_traj<2>(gr, dbuf[0], t0, dt, 0, s, ps.start, ps.stop, trig)
              : launch_traj<3>(gr, dbuf[0], t0, dt, 0, s, ps.start, ps.stop, trig);
    prof_end(gr, ps, 0, e);
    for (int k = 0; k < nsteps && e == hipSuccess; ++k) {
      gr->steps_launched++;
      sl::NextTraj nt{};
      if (k + 1 < nsteps) {
        nt.disp = dbuf[(k + 1) & 1];
        nt.st = stage_times(gr, t0 + (double)(k + 1) * dt, dt);
        nt.dt = dt;
        nt.integrator = gr->desc.integrator;
        nt.carried = carried ? 1 : 0;
        nt.trig = carried ? nullptr : trig;
      }
      e = reconstruct_launches(gr, ws, (k & 1) ? ba : ab, dbuf[k & 1], nt, s);
      if (e == hipSuccess) gr->reconstructs_launched++;
    }
    if (e == hipSuccess && result_in_b) *result_in_b = nsteps & 1;
    return hip_status(e);
  }
  void* const* cur = fields_a;
  void* const* nxt = fields_b;
  int in_b = 0;
  for (int s = 0; s < nsteps; s += K) {
    for (int k = 0; k < K; ++k) {
      if (gr->v.kind == SL_VEL_CARRIED) {
        // Straight lines with the velocity of the last reset (the fields `cur`).
        sl::FieldPtrs fp;
        int rc = field_ptrs(gr, (const void* const*)cur, nxt, &fp);
        if (rc != SL_OK) return rc;
        if (((uintptr_t)workspace) % kAlign) return SL_EINVAL;
        double* disp = reinterpret_cast<double*>(static_cast<char*>(workspace) + gr->off_disp);
        clear_stale_error();
        const ProfSlot ps = prof_begin(gr, 0);
        const hipStream_t hs = static_cast<hipStream_t>(stream);
        const hipError_t e =
            gr->desc.dim == 2 ? launch_carried<2>(gr, fp, disp, dt, k > 0, hs, ps.start, ps.stop)
                              : launch_carried<3>(gr, fp, disp, dt, k > 0, hs, ps.start, ps.stop);
        prof_end(gr, ps, 0, e);
        rc = hip_status(e);
        if (rc != SL_OK) return rc;
        gr->steps_since_reset++;
        gr->steps_launched++;
        continue;
      }
      const int rc = sl_step(gr, workspace, t0 + (double)(s + k) * dt, dt, stream);
      if (rc != SL_OK) return rc;
    }
    const int rc = sl_reconstruct(gr, workspace, (const void* const*)cur, nxt, stream);
    if (rc != SL_OK) return rc;
    void* const* tmp = cur;
    cur = nxt;
    nxt = tmp;
    in_b ^= 1;
  }
  if (result_in_b) *result_in_b = in_b;
  return SL_OK;
}

}  // extern "C"

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (with that device current).
int static_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_status(e);
  if (dev < 0 || dev >= kMaxDevices) return SL_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_status(e);
    if (!p) return SL_EHIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SL_OK;
}

}  // namespace

extern "C" {

int sl_advance_static(sl_grid* gr, void* const* fields_a, void* const* fields_b, double t0,
                      double dt, int nsteps, void* stream, int* result_in_b,
                      int64_t* counters) {
  if (!gr) return SL_EINVAL;
  if (gr->ws_bytes > SL_STATIC_SCRATCH_BYTES) {
    snprintf(g_detail, sizeof(g_detail),
             "grid needs %zu workspace bytes; the static scratch holds %zu", gr->ws_bytes,
             (size_t)SL_STATIC_SCRATCH_BYTES);
    return SL_ETOOBIG;
  }
  void* ws = nullptr;
  int rc = static_scratch(&ws);
  if (rc != SL_OK) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto* stats = reinterpret_cast<unsigned long long*>(static_cast<char*>(ws) + gr->off_stats);
  clear_stale_error();
  sl::zero_kernel<<<4, 256, 0, s>>>(stats, sl::kStatWords);
  rc = hip_status(hipGetLastError());
  if (rc != SL_OK) return rc;
  // The grid's counters of launched steps belong to sl_sync's workspace.
  const int64_t steps0 = gr->steps_launched, recs0 = gr->reconstructs_launched;
  rc = sl_advance(gr, ws, fields_a, fields_b, t0, dt, nsteps, stream, result_in_b);
  gr->steps_launched = steps0;
  gr->reconstructs_launched = recs0;
  if (rc != SL_OK) return rc;
  if (counters) {
    sl::static_counters_kernel<<<1, 64, 0, s>>>(stats, counters);
    rc = hip_status(hipGetLastError());
  }
  return rc;
}

int sl_profile_enable(sl_grid* gr, int period) {
  if (!gr) return SL_EINVAL;
  gr->prof_period = period > 0 ? period : 0;
  gr->prof_count[0] = gr->prof_count[1] = gr->prof_count[2] = gr->prof_count[3] = 0;
  return SL_OK;
}

int sl_profile_read(sl_grid* gr, sl_profile* out) {
  if (!gr) return SL_EINVAL;
  prof_fold(gr);
  if (out) {
    out->traj_launches = gr->prof_n[0];
    out->traj_ms = gr->prof_ms[0];
    out->recon_launches = gr->prof_n[1];
    out->recon_ms = gr->prof_ms[1];
    out->orders_launches = gr->prof_n[2];
    out->orders_ms = gr->prof_ms[2];
    out->source_launches = gr->prof_n[3];
    out->source_ms = gr->prof_ms[3];
  }
  for (int k = 0; k < 4; ++k) {
    gr->prof_n[k] = 0;
    gr->prof_ms[k] = 0.0;
  }
  return SL_OK;
}

const double* sl_displacement(const sl_grid* gr, const void* workspace, int axis) {
  if (!gr || !workspace || axis < 0 || axis >= gr->desc.dim) return nullptr;
  return reinterpret_cast<const double*>(static_cast<const char*>(workspace) + gr->off_disp) +
         (size_t)axis * (size_t)gr->ntot;
}

const char* sl_strerror(int code) {
  switch (code) {
    case SL_OK: return "ok";
    case SL_EINVAL: return "invalid argument";
    case SL_ENOMEM: return "out of host memory";
    case SL_EHIP: return "HIP runtime error";
    case SL_ESEARCH: return "host element not found";
    case SL_ENEWTON: return "Newton iteration did not converge";
    case SL_ENONFINITE: return "non-finite reconstructed value";
    case SL_EBUSY: return "resources exhausted";
    case SL_ESTATE: return "call out of order";
    case SL_ENOTFOUND: return "unknown request";
    case SL_ETOOBIG: return "grid larger than the static scratch";
    default: return "unknown status";
  }
}

int sl_version(void) { return SL_VERSION; }

const char* sl_error_detail(void) { return g_detail; }

}  // extern "C"
