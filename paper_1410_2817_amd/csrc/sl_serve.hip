// Continuous batching of many independent 2-D advection problems on one GPU.
//
// The caller hands the server one device arena.  The server keeps a table of
// request descriptors at its start and sub-allocates each admitted request's
// two field sets and lattice displacement from the rest (first fit, 256-byte
// aligned); a request that does not fit is refused with SL_EBUSY, so the
// arena size is the HBM budget.  Every tick advances each active request by
// one step of the scheme (trajectories, then reconstruction with the lattice
// reset) through batched reconstruction launches, one per (precision, field
// count), that also integrate each request's next-step trajectories into its
// other displacement buffer; only a request's first step needs a batched
// trajectory launch (one per velocity family).  Workgroups find
// their request from per-tick block offsets passed in the kernel arguments and
// run exactly the per-tile code of the single-grid kernels, so a request's
// result does not depend on what it was batched with.  Requests join between
// ticks as memory frees up and leave when their step count is reached.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <deque>
#include <map>
#include <new>
#include <vector>

#include "sl.h"
#include "sl_device.h"
#include "sl_grid.h"
#include "sl_launch.h"
#include "sl_recon2d.h"
#include "sl_traj.h"

namespace sl {

// Device-resident, written once at admission.
struct ReqStatic {
  GridArgs g;
  VelArgs v;
  FieldPtrs ab;  // in = set A, out = set B; odd steps swap them
  double* disp;   // displacement of even steps
  double* disp2;  // displacement of odd steps
  unsigned long long* stats;
  int tiles_x, ntiles;    // reconstruction tiles
  int traj_bx, traj_by;   // trajectory blocks (64 x 4 nodes each)
  int integrator;
  int pad;
  const double* trig;  // per-axis sin/cos table (sl::trig_table_kernel), or null
};

// Per tick and request, passed in the kernel arguments.
struct ReqTick {
  int entry;      // table index
  int blk_begin;  // first block of this request in the batched launch
  int parity;     // step parity: 0: A -> B from disp, 1: B -> A from disp2
  int next;       // reconstruction: also integrate the next step
  double dt;
  double tf[3];   // stage time factors (periodic velocity families) of the
                  // step the trajectories are for
};

constexpr int kServeBatch = 40;  // requests per batched launch (kernel-argument budget)

struct TickArgs {
  int nreq;
  int total_blocks;
  ReqTick r[kServeBatch];
};

// Request of batched block b (block offsets ascend; the search is uniform).
__device__ __forceinline__ int find_request(const TickArgs& ta, int b) {
  int i = 0;
  while (i + 1 < ta.nreq && ta.r[i + 1].blk_begin <= b) ++i;
  return i;
}

template <int VK>
__global__ __launch_bounds__(kBlock) void traj_batched_kernel(const ReqStatic* __restrict__ table,
                                                              TickArgs ta) {
  const int i = find_request(ta, blockIdx.x);
  const ReqTick& rt = ta.r[i];
  const ReqStatic& rs = table[rt.entry];
  const int lb = blockIdx.x - rt.blk_begin;
  const int bx = lb % rs.traj_bx, by = lb / rs.traj_bx;
  int idx[2] = {bx * kTrajBX + (int)(threadIdx.x % kTrajBX),
                by * kTrajBY + (int)(threadIdx.x / kTrajBX)};
  if (idx[0] >= rs.g.n[0] || idx[1] >= rs.g.n[1]) return;
  StageTimes st;
  st.tf[0] = rt.tf[0];
  st.tf[1] = rt.tf[1];
  st.tf[2] = rt.tf[2];
  st.tf[3] = rt.tf[2];
  traj_node<2, VK>(rs.g, rs.v, rs.disp, st, rt.dt, 0, rs.integrator, idx, rs.trig);
}

template <typename T, int NF>
__global__ __launch_bounds__(kTileThreads, (tile2d_waves<T, NF>()))
void recon2d_batched_kernel(
    const ReqStatic* __restrict__ table, TickArgs ta) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int logical = xcd_tile(blockIdx.x, ta.total_blocks);
  const int i = find_request(ta, logical);
  const ReqTick& rt = ta.r[i];
  const ReqStatic& rs = table[rt.entry];
  FieldPtrs fp;
#pragma unroll
  for (int f = 0; f < SL_MAX_FIELDS; ++f) {
    fp.in[f] = rt.parity ? rs.ab.out[f] : rs.ab.in[f];
    fp.out[f] = rt.parity ? const_cast<void*>(rs.ab.in[f]) : rs.ab.out[f];
  }
  NextTraj nt{};
  if (rt.next) {
    nt.disp = rt.parity ? rs.disp : rs.disp2;
    nt.st.tf[0] = rt.tf[0];
    nt.st.tf[1] = rt.tf[1];
    nt.st.tf[2] = rt.tf[2];
    nt.st.tf[3] = rt.tf[2];
    nt.dt = rt.dt;
    nt.integrator = rs.integrator;
    nt.trig = rs.trig;
  }
  recon2d_tile<T, NF>(rs.g, fp, rt.parity ? rs.disp2 : rs.disp, nullptr, rs.stats,
                      logical - rt.blk_begin, rs.tiles_x, smem, nt, rs.v);
}

// ---------------------------------------------------------------------------
// Multi-step serving kernel with a device-side work queue.
//
// One launch covers `window` ticks of every resident request whose values are
// of type T and that has NF fields (NF <= kServeMaxNF; a kernel per field
// count keeps each one's registers those of the batched kernel).  Its work is
// a list of segments, one per (request, step), in tick order; the tiles of
// each segment are split into 8 contiguous chunks, one per XCD, and each XCD
// has its own queue: the concatenation of its chunks over the segments.  The
// launch has one workgroup per tile of the whole window.  A workgroup reads
// the XCD it runs on and takes the next tile of that XCD's queue through one
// atomic counter (the next non-empty queue once its own is empty) and finds
// its segment by a 64-way search of the queue's prefix sums, so a
// request's neighbouring tiles meet in one L2, and tiles are handed out in
// tick order whatever order the workgroups start in.
//
// Steps of one request depend on each other: step s reads the fields and the
// displacement that step s - 1 wrote, and writes into buffers step s - 1 read
// from.  Within a launch, a request's segments after its first wait for every
// tile of its previous segment: each finished tile of a segment that a later
// one waits for is published with an agent-scope release (its writes reach
// the memory all XCDs share) and a count in `done`; the waiting workgroup
// acquires once the count has reached the segment's `need`.  A request's
// first segment of a launch needs no wait (the launch boundary orders it
// after the previous launch), so a one-tick launch has neither waits nor
// fences.  Every queue hands out its tiles in tick order and a tile only
// waits for tiles of earlier segments, which were handed to workgroups that
// are already running, so the waits always end.  A wait that still exceeds
// kServeSpinLimit polls (a failure elsewhere) sets `abort`; every workgroup
// that sees it leaves, and the host reports SL_EHIP.
//
// (A fixed grid of workgroups that loop over the queue was tried first: with
// the tile code inside a loop the compiler could no longer keep the
// request's parameters in scalar registers and spilled about 60 VGPRs per
// lane, so each workgroup takes one tile.)

constexpr int kServeMaxNF = 4;  // field counts the window kernels take
constexpr unsigned kServeSpinLimit = 1u << 23;
// Queue counters sit 256 bytes apart: atomics on one line serialise.
constexpr int kQueueStride = 64;

struct ServeSeg {
  int entry;   // table index
  int parity;  // 0: A -> B from disp, 1: B -> A from disp2
  int next;    // also integrate the next step's trajectories
  int ntiles;
  unsigned need;  // published tiles of the request before this segment starts
  int wait;       // 1: wait for `need` (not the request's first segment here)
  int publish;    // 1: a later segment of this launch waits for these tiles
  double dt;
  double tf[3];  // stage time factors of the next step's trajectories
};

__device__ __forceinline__ int xcc_id() {
  // HW_REG_XCC_ID (register 20), bits [3:0]: the XCD this wave runs on.
  return (int)(__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & (kNumXcd - 1));
}

template <typename T, int NF>
__device__ __forceinline__ void serve_tile(const ReqStatic& rs, const ServeSeg& sg, int tile,
                                           unsigned char* smem) {
  FieldPtrs fp;
#pragma unroll
  for (int f = 0; f < SL_MAX_FIELDS; ++f) {
    fp.in[f] = sg.parity ? rs.ab.out[f] : rs.ab.in[f];
    fp.out[f] = sg.parity ? const_cast<void*>(rs.ab.in[f]) : rs.ab.out[f];
  }
  NextTraj nt{};
  if (sg.next) {
    nt.disp = sg.parity ? rs.disp : rs.disp2;
    nt.st.tf[0] = sg.tf[0];
    nt.st.tf[1] = sg.tf[1];
    nt.st.tf[2] = sg.tf[2];
    nt.st.tf[3] = sg.tf[2];
    nt.dt = sg.dt;
    nt.integrator = rs.integrator;
    nt.trig = rs.trig;
  }
  recon2d_tile<T, NF>(rs.g, fp, sg.parity ? rs.disp2 : rs.disp, nullptr, rs.stats, tile,
                      rs.tiles_x, smem, nt, rs.v);
}

template <typename T, int NF>
__global__ __launch_bounds__(kTileThreads, (tile2d_waves<T, NF>()))
void serve_window_kernel(const ReqStatic* __restrict__ table,
                         const ServeSeg* __restrict__ segs,
                         const int* __restrict__ prefix,  // kNumXcd x (nseg + 1)
                         int nseg, unsigned* __restrict__ qctr,
                         unsigned* __restrict__ done, int* __restrict__ abort_flag) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_item, s_seg, s_x;
  if (threadIdx.x < 64) {
    // Wave 0 takes the workgroup's tile: lane 0 the atomic, all 64 lanes the
    // search for its segment (a 64-way split of the prefix per round).
    const int lane = threadIdx.x;
    const int home = xcc_id();
    int it = 0, k = -1, x = home;
    if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
      for (int q = 0; q < kNumXcd && k < 0; ++q) {
        x = (home + q) & (kNumXcd - 1);
        const int* __restrict__ pre = prefix + x * (nseg + 1);
        const int total = pre[nseg];
        unsigned* ctr = qctr + x * kQueueStride;
        int got = total;
        if (lane == 0 &&
            __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < (unsigned)total)
          got = (int)atomicAdd(ctr, 1u);
        it = __builtin_amdgcn_readfirstlane(got);
        if (it >= total) continue;  // drained
        int lo = 0, hi = nseg;  // pre[lo] <= it < pre[hi]
        while (hi - lo > 1) {
          const int step = (hi - lo + 63) >> 6;
          const int idx = min(lo + lane * step, hi - 1);
          const unsigned long long below = __ballot(pre[idx] <= it);
          const int top = 63 - __builtin_clzll(below);  // lane 0 always qualifies
          const int nlo = min(lo + top * step, hi - 1);
          const int nhi = top < 63 ? min(lo + (top + 1) * step, hi) : hi;
          lo = nlo;
          hi = nhi;
        }
        k = lo;
      }
    }
    if (lane == 0 && k >= 0 && segs[k].wait) {
      const ServeSeg& sg = segs[k];
      unsigned spins = 0;
      while (__hip_atomic_load(&done[sg.entry], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
             sg.need) {
        if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
            ++spins > kServeSpinLimit) {
          __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          k = -1;
          break;
        }
        __builtin_amdgcn_s_sleep(4);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    if (lane == 0) {
      s_item = it;
      s_seg = k;
      s_x = x;
    }
  }
  __syncthreads();
  // Uniform across the workgroup: keep them (and what is loaded through
  // them) in scalar registers.
  const int k = __builtin_amdgcn_readfirstlane(s_seg);
  if (k < 0) return;
  const int it = __builtin_amdgcn_readfirstlane(s_item);
  const int x = __builtin_amdgcn_readfirstlane(s_x);
  const ServeSeg& sg = segs[k];
  const ReqStatic& rs = table[sg.entry];
  const int tile = sg.ntiles * x / kNumXcd + (it - prefix[x * (nseg + 1) + k]);
  serve_tile<T, NF>(rs, sg, tile, smem);
  if (sg.publish) {
    __syncthreads();
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_fetch_add(&done[sg.entry], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

__global__ void serve_zero_kernel(unsigned* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    p[i] = 0u;
}

}  // namespace sl

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Request {
  int64_t id;
  int entry;
  sl_grid* grid;
  size_t off, bytes;
  int nsteps, done;
  double t0, dt;
  int64_t finish_tick;
  bool reported;
  unsigned published;  // tiles counted in the device's done[entry] (window launches)
  void* a[SL_MAX_FIELDS];
  void* b[SL_MAX_FIELDS];
};

constexpr int kServeMaxWindow = 16;  // ticks per window launch
// Window kernels: one per value precision and field count 1..kServeMaxNF;
// group = precision * kServeMaxNF + nf - 1.
constexpr int kServeGroups = 2 * sl::kServeMaxNF;

// Bytes of a tick's upload for the window kernels: the queue counters of
// every group (zeros, kQueueStride apart), the segments, the per-XCD prefix
// sums.
constexpr size_t kQueueBytes =
    sizeof(unsigned) * kServeGroups * sl::kNumXcd * sl::kQueueStride;

inline size_t tick_area_bytes(int max_requests) {
  const size_t max_segs = (size_t)max_requests * kServeMaxWindow;
  return kQueueBytes + (sizeof(sl::ServeSeg) * max_segs + 255) / 256 * 256 +
         (sizeof(int) * sl::kNumXcd * (max_segs + kServeGroups) + 255) / 256 * 256;
}

// Host staging of one window launch's segment table (pinned memory).
struct SegStage {
  char* base;  // queue counters (zeros), then the segments, then the prefix sums
};

}  // namespace

struct sl_server {
  char* arena;
  size_t arena_bytes;
  hipStream_t stream;
  int max_requests;
  int max_inflight;
  sl::ReqStatic* table;                 // device, at the arena start
  std::vector<sl::ReqStatic> host_table;  // host copies (stable source of the uploads)
  unsigned long long* stats;            // device counters shared by all requests
  std::map<size_t, size_t> free_blocks;   // offset -> size
  std::vector<int> free_entries;
  std::vector<Request> active;
  std::vector<Request> finished;
  int64_t next_id;
  int64_t tick;
  std::deque<std::pair<int64_t, hipEvent_t>> tick_events;
  std::vector<hipEvent_t> ev_pool;
  int64_t completed_tick;
  size_t in_use;
  // Launch mode of sl_server_tick (sl_server_set_mode).
  int mode;
  int window;
  // Window launches: the device segment table of a tick (the groups of
  // one value precision and field count one after another) and its per-XCD
  // prefix sums, per-group queue counters, per-entry published-tile counts
  // and the abort flag, all in the arena header; pinned host staging, one
  // slot per tick in flight.
  char* dev_tick;   // a tick's queue counters, segments and prefix sums (one upload)
  unsigned* done;  // max_requests
  int* abort_flag;
  std::vector<SegStage> stage;
  void* stage_mem;
  std::vector<sl::ServeSeg> segs;  // host scratch of a tick's segments
  std::vector<int> prefix;         // and of their per-XCD prefix sums
  // Host totals since the last sl_server_sync.
  int64_t stat_nodes, stat_steps;
};

namespace {

bool arena_alloc(sl_server* s, size_t bytes, size_t* off) {
  for (auto it = s->free_blocks.begin(); it != s->free_blocks.end(); ++it) {
    if (it->second >= bytes) {
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t roff = it->first + bytes;
      s->free_blocks.erase(it);
      if (rest) s->free_blocks[roff] = rest;
      s->in_use += bytes;
      return true;
    }
  }
  return false;
}

void arena_free(sl_server* s, size_t off, size_t bytes) {
  auto it = s->free_blocks.emplace(off, bytes).first;
  // Coalesce with the following block, then with the preceding one.
  auto nx = std::next(it);
  if (nx != s->free_blocks.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    s->free_blocks.erase(nx);
  }
  if (it != s->free_blocks.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      s->free_blocks.erase(it);
    }
  }
  s->in_use -= bytes;
}

size_t request_bytes(const sl_grid* gr) {
  const size_t vbytes = gr->desc.value_prec == SL_FP32 ? 4 : 8;
  const size_t field = align_up(vbytes * (size_t)gr->ntot);
  // The batched reconstruction evaluates the limiter flags in LDS, so the
  // request needs the workspace only up to the order-word arrays, plus the
  // second displacement buffer and the trajectories' sin/cos table.
  return 2 * (size_t)gr->desc.nfields * field + align_up(gr->off_ord) +
         align_up(sizeof(double) * 2 * (size_t)gr->ntot) + align_up(gr->trig_bytes);
}

hipEvent_t take_event(sl_server* s) {
  if (!s->ev_pool.empty()) {
    hipEvent_t e = s->ev_pool.back();
    s->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  return e;
}

// Mark finished ticks (events that have completed), oldest first.
void drain_events(sl_server* s, bool wait_all, size_t keep) {
  while (!s->tick_events.empty()) {
    hipEvent_t e = s->tick_events.front().second;
    const bool must_wait = wait_all || s->tick_events.size() > keep;
    if (must_wait) {
      if (hipEventSynchronize(e) != hipSuccess) break;
    } else if (hipEventQuery(e) != hipSuccess) {
      break;
    }
    s->completed_tick = s->tick_events.front().first;
    s->ev_pool.push_back(e);
    s->tick_events.pop_front();
  }
}

template <typename T>
hipError_t launch_recon_group(sl_server* s, int nf, const sl::TickArgs& ta) {
  const dim3 grid(ta.total_blocks), block(sl::kTileThreads);
#define SL_SERVE_RECON(NF)                                                               \
  case NF:                                                                               \
    return sl::launch(sl::recon2d_batched_kernel<T, NF>, grid, block,                   \
                      (uint32_t)sl::Tile2D<T, NF>::LDS_BYTES, s->stream, nullptr, nullptr, \
                      (const sl::ReqStatic*)s->table, ta);
  switch (nf) {
    SL_SERVE_RECON(1)
    SL_SERVE_RECON(2)
    SL_SERVE_RECON(3)
    SL_SERVE_RECON(4)
    SL_SERVE_RECON(5)
    SL_SERVE_RECON(6)
    SL_SERVE_RECON(7)
    default:
      return sl::launch(sl::recon2d_batched_kernel<T, 8>, grid, block,
                        (uint32_t)sl::Tile2D<T, 8>::LDS_BYTES, s->stream, nullptr, nullptr,
                        (const sl::ReqStatic*)s->table, ta);
  }
#undef SL_SERVE_RECON
}

hipError_t launch_traj_group(sl_server* s, int vk, const sl::TickArgs& ta) {
  const dim3 grid(ta.total_blocks), block(sl::kBlock);
  const sl::ReqStatic* t = s->table;
  switch (vk) {
    case SL_VEL_UNIFORM:
      return sl::launch(sl::traj_batched_kernel<SL_VEL_UNIFORM>, grid, block, 0, s->stream, nullptr, nullptr, t, ta);
    case SL_VEL_SOLID_BODY:
      return sl::launch(sl::traj_batched_kernel<SL_VEL_SOLID_BODY>, grid, block, 0, s->stream, nullptr, nullptr, t, ta);
    case SL_VEL_SWIRL2D:
      return sl::launch(sl::traj_batched_kernel<SL_VEL_SWIRL2D>, grid, block, 0, s->stream, nullptr, nullptr, t, ta);
    default:
      return sl::launch(sl::traj_batched_kernel<SL_VEL_FOURIER>, grid, block, 0, s->stream, nullptr, nullptr, t, ta);
  }
}

// The window kernel of group `grp` (value precision * kServeMaxNF + field
// count - 1) and its dynamic LDS bytes.
struct WindowKernel {
  const void* fn;
  uint32_t lds;
};

template <typename T, int NF>
WindowKernel window_kernel_of() {
  return {reinterpret_cast<const void*>(sl::serve_window_kernel<T, NF>),
          (uint32_t)sl::Tile2D<T, NF>::LDS_BYTES};
}

WindowKernel window_kernel(int grp) {
  static_assert(sl::kServeMaxNF == 4, "one case per field count");
  switch (grp) {
    case 0: return window_kernel_of<double, 1>();
    case 1: return window_kernel_of<double, 2>();
    case 2: return window_kernel_of<double, 3>();
    case 3: return window_kernel_of<double, 4>();
    case 4: return window_kernel_of<float, 1>();
    case 5: return window_kernel_of<float, 2>();
    case 6: return window_kernel_of<float, 3>();
    default: return window_kernel_of<float, 4>();
  }
}

// Group `grp`'s window kernel over `tiles` tiles (one workgroup each).
hipError_t launch_window(sl_server* s, int grp, const sl::ServeSeg* segs, const int* prefix,
                         int nseg, int tiles, unsigned* qctr) {
  const WindowKernel wk = window_kernel(grp);
  const sl::ReqStatic* table = s->table;
  void* args[] = {&table, &segs, &prefix, &nseg, &qctr, &s->done, &s->abort_flag};
  return hipExtLaunchKernel(wk.fn, dim3((unsigned)tiles), dim3(sl::kTileThreads), args, wk.lds,
                            s->stream, nullptr, nullptr, 0);
}

// Stage time factors of step `k` of request r.
void stage_times(const Request& r, int k, double tf[3]) {
  const sl_grid* gr = r.grid;
  const double t = r.t0 + (double)k * r.dt, dt = r.dt;
  const bool periodic = gr->v.kind == SL_VEL_SWIRL2D;
  const bool rk4 = gr->desc.integrator == SL_RK4;
  const double ts[3] = {t, rk4 ? t + 0.5 * dt : t + dt / 3.0, rk4 ? t + dt : t + 0.75 * dt};
  for (int i = 0; i < 3; ++i) tf[i] = periodic ? cos(M_PI * ts[i] / gr->v.p[0]) : 1.0;
}

}  // namespace

extern "C" {

size_t sl_server_arena_overhead(int max_requests) {
  if (max_requests < 1 || max_requests > 4096) return 0;
  return align_up(sizeof(sl::ReqStatic) * (size_t)max_requests) +
         align_up(sizeof(unsigned long long) * sl::kStatWords) + tick_area_bytes(max_requests) +
         align_up(sizeof(unsigned) * (size_t)max_requests + sizeof(int));
}

size_t sl_server_request_bytes(const sl_grid_desc* desc) {
  sl_grid* gr = nullptr;
  if (sl_create_grid(desc, &gr) != SL_OK) return 0;
  const size_t b = request_bytes(gr);
  sl_destroy_grid(gr);
  return b;
}

int sl_server_create(void* arena, size_t arena_bytes, int max_requests, int max_inflight,
                     void* stream, sl_server** out) {
  if (!out) return SL_EINVAL;
  *out = nullptr;
  if (!arena || ((uintptr_t)arena) % kAlign || max_requests < 1 || max_requests > 4096 ||
      max_inflight < 1)
    return SL_EINVAL;
  const size_t table_bytes = align_up(sizeof(sl::ReqStatic) * (size_t)max_requests);
  const size_t stats_bytes = align_up(sizeof(unsigned long long) * sl::kStatWords);
  const size_t tick_bytes = tick_area_bytes(max_requests);
  const size_t ctl_bytes = align_up(sizeof(unsigned) * (size_t)max_requests + sizeof(int));
  const size_t persist_bytes = tick_bytes + ctl_bytes;
  if (arena_bytes < sl_server_arena_overhead(max_requests) + kAlign) return SL_EINVAL;
  sl_server* s = new (std::nothrow) sl_server();
  if (!s) return SL_ENOMEM;
  s->arena = static_cast<char*>(arena);
  s->arena_bytes = arena_bytes;
  s->stream = static_cast<hipStream_t>(stream);
  s->max_requests = max_requests;
  s->max_inflight = max_inflight;
  s->table = reinterpret_cast<sl::ReqStatic*>(s->arena);
  s->stats = reinterpret_cast<unsigned long long*>(s->arena + table_bytes);
  s->host_table.resize(max_requests);
  char* ph = s->arena + table_bytes + stats_bytes;
  s->dev_tick = ph;
  s->done = reinterpret_cast<unsigned*>(ph + tick_bytes);
  s->abort_flag = reinterpret_cast<int*>(s->done + max_requests);
  s->mode = SL_SERVE_BATCHED;
  s->window = 1;
  s->stage_mem = nullptr;
  s->stat_nodes = s->stat_steps = 0;
  const size_t heap = table_bytes + stats_bytes + persist_bytes;
  s->free_blocks[heap] = (arena_bytes - heap) / kAlign * kAlign;
  for (int e = max_requests - 1; e >= 0; --e) s->free_entries.push_back(e);
  s->next_id = 1;
  s->tick = 0;
  s->completed_tick = 0;
  s->in_use = 0;
  // Counters, queue counters, published counts and the abort flag start at
  // zero.
  int rc = SL_OK;
  {
    sl::serve_zero_kernel<<<8, 256, 0, s->stream>>>(reinterpret_cast<unsigned*>(s->stats),
                                                   2 * sl::kStatWords);
    const int nctl = (int)(ctl_bytes / sizeof(unsigned));
    sl::serve_zero_kernel<<<(nctl + 255) / 256, 256, 0, s->stream>>>(s->done, nctl);
    if (hipGetLastError() != hipSuccess) rc = SL_EHIP;
  }
  if (rc == SL_OK) {
    const size_t slot = tick_bytes;
    const int nslots = max_inflight + 1;
    if (hipHostMalloc(&s->stage_mem, slot * (size_t)nslots, hipHostMallocDefault) != hipSuccess)
      rc = SL_EHIP;
    for (int k = 0; k < nslots && rc == SL_OK; ++k) {
      s->stage.push_back({static_cast<char*>(s->stage_mem) + slot * (size_t)k});
    }
  }
  if (rc != SL_OK) {
    (void)hipStreamSynchronize(s->stream);
    if (s->stage_mem) (void)hipHostFree(s->stage_mem);
    delete s;
    return rc;
  }
  *out = s;
  return SL_OK;
}

int sl_server_destroy(sl_server* s) {
  if (!s) return SL_OK;
  (void)hipStreamSynchronize(s->stream);
  for (auto& p : s->tick_events) s->ev_pool.push_back(p.second);
  for (hipEvent_t e : s->ev_pool) (void)hipEventDestroy(e);
  for (auto& r : s->active) sl_destroy_grid(r.grid);
  for (auto& r : s->finished) sl_destroy_grid(r.grid);
  if (s->stage_mem) (void)hipHostFree(s->stage_mem);
  delete s;
  return SL_OK;
}

int sl_server_admit(sl_server* s, const sl_grid_desc* desc, const void* const* fields_in,
                    double t0, double dt, int nsteps, int64_t* id) {
  if (!s || !desc || !fields_in || !id || nsteps < 1 || !isfinite(t0) || !isfinite(dt))
    return SL_EINVAL;
  if (desc->dim != 2 || desc->reconstruct_every != 1) return SL_EINVAL;
  if (desc->vel.kind == SL_VEL_DEFORM3D || desc->vel.kind == SL_VEL_GRIDDED ||
      desc->vel.kind == SL_VEL_CARRIED)
    return SL_EINVAL;
  sl_grid* gr = nullptr;
  int rc = sl_create_grid(desc, &gr);
  if (rc != SL_OK) return rc;
  for (int f = 0; f < desc->nfields; ++f)
    if (!fields_in[f]) {
      sl_destroy_grid(gr);
      return SL_EINVAL;
    }
  if (s->free_entries.empty()) {
    sl_destroy_grid(gr);
    return SL_EBUSY;
  }
  const size_t bytes = request_bytes(gr);
  size_t off = 0;
  if (!arena_alloc(s, bytes, &off)) {
    sl_destroy_grid(gr);
    return SL_EBUSY;
  }
  Request r;
  memset(&r, 0, sizeof(r));
  r.id = s->next_id++;
  r.entry = s->free_entries.back();
  s->free_entries.pop_back();
  r.grid = gr;
  r.off = off;
  r.bytes = bytes;
  r.nsteps = nsteps;
  r.t0 = t0;
  r.dt = dt;
  r.finish_tick = -1;
  const size_t vbytes = desc->value_prec == SL_FP32 ? 4 : 8;
  const size_t field = align_up(vbytes * (size_t)gr->ntot);
  char* base = s->arena + off;
  for (int f = 0; f < desc->nfields; ++f) {
    r.a[f] = base + (size_t)f * field;
    r.b[f] = base + (size_t)(desc->nfields + f) * field;
  }
  char* ws = base + 2 * (size_t)desc->nfields * field;

  sl::ReqStatic& hs = s->host_table[r.entry];
  memset(&hs, 0, sizeof(hs));
  hs.g = gr->g;
  hs.v = gr->v;
  for (int f = 0; f < desc->nfields; ++f) {
    hs.ab.in[f] = r.a[f];
    hs.ab.out[f] = r.b[f];
  }
  hs.disp = reinterpret_cast<double*>(ws + gr->off_disp);
  hs.disp2 = reinterpret_cast<double*>(ws + align_up(gr->off_ord));
  double* trig = gr->trig_bytes ? reinterpret_cast<double*>(
                                      ws + align_up(gr->off_ord) +
                                      align_up(sizeof(double) * 2 * (size_t)gr->ntot))
                                : nullptr;
  hs.trig = trig;
  hs.stats = s->stats;
  using C = sl::Tile2D<float, 1>;
  hs.tiles_x = (gr->g.n[0] + C::TX - 1) / C::TX;
  hs.ntiles = hs.tiles_x * ((gr->g.n[1] + C::TY - 1) / C::TY);
  hs.traj_bx = (gr->g.n[0] + sl::kTrajBX - 1) / sl::kTrajBX;
  hs.traj_by = (gr->g.n[1] + sl::kTrajBY - 1) / sl::kTrajBY;
  hs.integrator = desc->integrator;

  hipError_t e = hipMemcpyAsync(s->table + r.entry, &hs, sizeof(hs), hipMemcpyHostToDevice,
                                s->stream);
  if (e == hipSuccess) {
    // The entry's published-tile count restarts (window launches).
    sl::serve_zero_kernel<<<1, 64, 0, s->stream>>>(s->done + r.entry, 1);
    e = hipGetLastError();
  }
  if (e == hipSuccess && trig) e = sl::launch_trig_table<2>(gr->g, gr->v, trig, s->stream);
  for (int f = 0; f < desc->nfields && e == hipSuccess; ++f)
    e = hipMemcpyAsync(r.a[f], fields_in[f], vbytes * (size_t)gr->ntot,
                       hipMemcpyDeviceToDevice, s->stream);
  if (e != hipSuccess) {
    arena_free(s, off, bytes);
    s->free_entries.push_back(r.entry);
    sl_destroy_grid(gr);
    return SL_EHIP;
  }
  s->active.push_back(r);
  *id = r.id;
  return SL_OK;
}

int sl_server_tick(sl_server* s, int* active) {
  if (!s) return SL_EINVAL;
  if (active) *active = (int)s->active.size();
  if (s->active.empty()) return SL_OK;
  // Keep at most max_inflight ticks queued on the device.
  drain_events(s, false, (size_t)s->max_inflight - 1);

  // First-step trajectories of newly admitted requests, batched per velocity
  // family (later steps' come from the previous tick's reconstruction).
  std::vector<int> order;
  for (size_t i = 0; i < s->active.size(); ++i)
    if (s->active[i].done == 0) order.push_back((int)i);
  auto vk_of = [&](int i) { return s->active[i].grid->v.kind; };
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return vk_of(x) < vk_of(y); });
  hipError_t err = hipSuccess;
  for (size_t i = 0; i < order.size() && err == hipSuccess;) {
    const int vk = vk_of(order[i]);
    sl::TickArgs ta;
    memset(&ta, 0, sizeof(ta));
    int blocks = 0;
    while (i < order.size() && vk_of(order[i]) == vk && ta.nreq < sl::kServeBatch) {
      const Request& r = s->active[order[i]];
      const sl::ReqStatic& hs = s->host_table[r.entry];
      sl::ReqTick& rt = ta.r[ta.nreq++];
      rt.entry = r.entry;
      rt.blk_begin = blocks;
      rt.parity = 0;
      rt.dt = r.dt;
      stage_times(r, 0, rt.tf);
      blocks += hs.traj_bx * hs.traj_by;
      ++i;
    }
    ta.total_blocks = blocks;
    err = launch_traj_group(s, vk, ta);
  }
  // Steps of each request this tick: up to `window` for the requests the
  // window kernels take, one for the others.
  const bool windowed = s->mode == SL_SERVE_QUEUED;
  auto in_window = [&](const Request& r) {
    return windowed && r.grid->desc.nfields <= sl::kServeMaxNF;
  };
  std::vector<int> nstep(s->active.size(), 1);
  for (size_t i = 0; i < s->active.size(); ++i) {
    const Request& r = s->active[i];
    if (in_window(r)) nstep[i] = std::min(s->window, r.nsteps - r.done);
  }
  // Window launches, one per (value precision, field count) group; the
  // tick's segment table holds the groups one after another.
  if (windowed && err == hipSuccess) {
    SegStage& st = s->stage[(size_t)(s->tick % (int64_t)s->stage.size())];
    std::vector<sl::ServeSeg>& segs = s->segs;
    std::vector<int>& prefix = s->prefix;
    segs.clear();
    prefix.clear();
    int seg0[kServeGroups + 1], pre0[kServeGroups + 1], tiles[kServeGroups];
    for (int grp = 0; grp < kServeGroups; ++grp) {
      const int prec = grp / sl::kServeMaxNF, nf = grp % sl::kServeMaxNF + 1;
      auto member = [&](const Request& r) {
        return in_window(r) && r.grid->desc.value_prec == prec &&
               r.grid->desc.nfields == nf;
      };
      seg0[grp] = (int)segs.size();
      pre0[grp] = (int)prefix.size();
      int maxw = 0;
      for (size_t i = 0; i < s->active.size(); ++i)
        if (member(s->active[i])) maxw = std::max(maxw, nstep[i]);
      // Tick-major order: every queue hands out a request's steps in order.
      for (int j = 0; j < maxw; ++j)
        for (size_t i = 0; i < s->active.size(); ++i) {
          const Request& r = s->active[i];
          if (!member(r) || j >= nstep[i]) continue;
          const sl::ReqStatic& hs = s->host_table[r.entry];
          sl::ServeSeg sg;
          const int step = r.done + j;
          sg.entry = r.entry;
          sg.parity = step & 1;
          sg.next = step + 1 < r.nsteps;
          sg.ntiles = hs.ntiles;
          sg.wait = j > 0;
          sg.need = r.published + (unsigned)j * (unsigned)hs.ntiles;
          sg.publish = j + 1 < nstep[i];
          sg.dt = r.dt;
          sg.tf[0] = sg.tf[1] = sg.tf[2] = 1.0;
          if (sg.next) stage_times(r, step + 1, sg.tf);
          segs.push_back(sg);
        }
      const int n = (int)segs.size() - seg0[grp];
      tiles[grp] = 0;
      for (int k = seg0[grp]; k < (int)segs.size(); ++k) tiles[grp] += segs[k].ntiles;
      // Per-XCD prefix sums of the segments' chunk sizes.
      if (n > 0)
        for (int x = 0; x < sl::kNumXcd; ++x) {
          prefix.push_back(0);
          for (int k = 0; k < n; ++k) {
            const int t = segs[seg0[grp] + k].ntiles;
            prefix.push_back(prefix.back() + (t * (x + 1) / sl::kNumXcd - t * x / sl::kNumXcd));
          }
        }
    }
    seg0[kServeGroups] = (int)segs.size();
    pre0[kServeGroups] = (int)prefix.size();
    if (!segs.empty()) {
      // One upload: zeroed queue counters, the segments, the prefix sums.
      const size_t seg_off = kQueueBytes;
      const size_t pre_off = align_up(seg_off + sizeof(sl::ServeSeg) * segs.size());
      const size_t bytes = pre_off + sizeof(int) * prefix.size();
      memset(st.base, 0, kQueueBytes);
      memcpy(st.base + seg_off, segs.data(), sizeof(sl::ServeSeg) * segs.size());
      memcpy(st.base + pre_off, prefix.data(), sizeof(int) * prefix.size());
      err = hipMemcpyAsync(s->dev_tick, st.base, bytes, hipMemcpyHostToDevice, s->stream);
      const auto* dsegs = reinterpret_cast<const sl::ServeSeg*>(s->dev_tick + seg_off);
      const int* dpre = reinterpret_cast<const int*>(s->dev_tick + pre_off);
      auto* dq = reinterpret_cast<unsigned*>(s->dev_tick);
      for (int grp = 0; grp < kServeGroups && err == hipSuccess; ++grp) {
        const int n = seg0[grp + 1] - seg0[grp];
        if (n > 0)
          err = launch_window(s, grp, dsegs + seg0[grp], dpre + pre0[grp], n, tiles[grp],
                              dq + grp * sl::kNumXcd * sl::kQueueStride);
      }
    }
  }
  // The other requests: one batched reconstruction launch per (value
  // precision, field count).
  order.clear();
  for (size_t i = 0; i < s->active.size(); ++i)
    if (!in_window(s->active[i])) order.push_back((int)i);
  auto key_of = [&](int i) {
    const sl_grid* g = s->active[i].grid;
    return g->desc.value_prec * 16 + g->desc.nfields;
  };
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return key_of(x) < key_of(y); });
  for (size_t i = 0; i < order.size() && err == hipSuccess;) {
    const int key = key_of(order[i]);
    sl::TickArgs ta;
    memset(&ta, 0, sizeof(ta));
    int blocks = 0;
    while (i < order.size() && key_of(order[i]) == key && ta.nreq < sl::kServeBatch) {
      const Request& r = s->active[order[i]];
      const sl::ReqStatic& hs = s->host_table[r.entry];
      sl::ReqTick& rt = ta.r[ta.nreq++];
      rt.entry = r.entry;
      rt.blk_begin = blocks;
      rt.parity = r.done & 1;
      rt.next = r.done + 1 < r.nsteps;
      rt.dt = r.dt;
      if (rt.next) stage_times(r, r.done + 1, rt.tf);
      blocks += hs.ntiles;
      ++i;
    }
    ta.total_blocks = blocks;
    const int nf = key % 16;
    err = (key / 16 == SL_FP32) ? launch_recon_group<float>(s, nf, ta)
                                : launch_recon_group<double>(s, nf, ta);
  }
  if (err != hipSuccess) return SL_EHIP;
  ++s->tick;
  hipEvent_t ev = take_event(s);
  if (!ev || hipEventRecord(ev, s->stream) != hipSuccess) return SL_EHIP;
  s->tick_events.emplace_back(s->tick, ev);
  // Advance the step counters; move completed requests out of the batch.
  std::vector<Request> still;
  still.reserve(s->active.size());
  for (size_t i = 0; i < s->active.size(); ++i) {
    Request& r = s->active[i];
    const int n = nstep[i];
    if (in_window(r)) r.published += (unsigned)(n - 1) * (unsigned)s->host_table[r.entry].ntiles;
    r.done += n;
    s->stat_nodes += (int64_t)n * r.grid->ntot;
    s->stat_steps += n;
    if (r.done >= r.nsteps) {
      r.finish_tick = s->tick;
      s->finished.push_back(r);
    } else {
      still.push_back(r);
    }
  }
  s->active.swap(still);
  if (active) *active = (int)s->active.size();
  return SL_OK;
}

int sl_server_set_mode(sl_server* s, int mode, int window) {
  if (!s || (mode != SL_SERVE_BATCHED && mode != SL_SERVE_QUEUED) || window < 1 ||
      window > kServeMaxWindow || (mode == SL_SERVE_BATCHED && window != 1))
    return SL_EINVAL;
  s->mode = mode;
  s->window = window;
  return SL_OK;
}

int sl_server_poll(sl_server* s, int64_t* done_ids, int max_ids, int* ndone) {
  if (!s || !ndone || max_ids < 0 || (max_ids > 0 && !done_ids)) return SL_EINVAL;
  drain_events(s, false, (size_t)-1);
  int n = 0;
  for (Request& r : s->finished) {
    if (n >= max_ids) break;
    if (!r.reported && r.finish_tick <= s->completed_tick) {
      r.reported = true;
      done_ids[n++] = r.id;
    }
  }
  *ndone = n;
  return SL_OK;
}

int sl_server_fetch(sl_server* s, int64_t id, void* const* fields_out) {
  if (!s || !fields_out) return SL_EINVAL;
  for (size_t i = 0; i < s->finished.size(); ++i) {
    Request& r = s->finished[i];
    if (r.id != id) continue;
    const int nf = r.grid->desc.nfields;
    const size_t vbytes = r.grid->desc.value_prec == SL_FP32 ? 4 : 8;
    void* const* res = (r.nsteps & 1) ? r.b : r.a;
    for (int f = 0; f < nf; ++f) {
      if (!fields_out[f]) return SL_EINVAL;
      if (hipMemcpyAsync(fields_out[f], res[f], vbytes * (size_t)r.grid->ntot,
                         hipMemcpyDeviceToDevice, s->stream) != hipSuccess)
        return SL_EHIP;
    }
    // Later work on the stream runs after the copy, so the memory can be
    // handed to the next admission right away.
    arena_free(s, r.off, r.bytes);
    s->free_entries.push_back(r.entry);
    sl_destroy_grid(r.grid);
    s->finished.erase(s->finished.begin() + (long)i);
    return SL_OK;
  }
  return SL_ENOTFOUND;
}

int sl_server_sync(sl_server* s, sl_stats* out) {
  if (!s) return SL_EINVAL;
  unsigned long long copies[sl::kStatWords], host[sl::ST_COUNT];
  int aborted = 0;
  if (hipMemcpyAsync(copies, s->stats, sizeof(copies), hipMemcpyDeviceToHost, s->stream) !=
          hipSuccess ||
      hipMemcpyAsync(&aborted, s->abort_flag, sizeof(int), hipMemcpyDeviceToHost, s->stream) !=
          hipSuccess)
    return SL_EHIP;
  sl::serve_zero_kernel<<<8, 256, 0, s->stream>>>(reinterpret_cast<unsigned*>(s->stats),
                                                 2 * sl::kStatWords);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s->stream) != hipSuccess)
    return SL_EHIP;
  sl::stat_totals(copies, host);
  drain_events(s, true, 0);
  if (out) {
    memset(out, 0, sizeof(*out));
    out->nodes = s->stat_nodes;
    out->search_fail = (int64_t)host[sl::ST_SEARCH_FAIL];
    out->newton_fail = (int64_t)host[sl::ST_NEWTON_FAIL];
    out->nonfinite = (int64_t)host[sl::ST_NONFINITE];
    out->order_hist[0] = (int64_t)host[sl::ST_ORDER0];
    out->order_hist[1] = (int64_t)host[sl::ST_ORDER1];
    out->order_hist[2] = (int64_t)host[sl::ST_ORDER2];
    out->walked = (int64_t)host[sl::ST_WALKED];
    out->scanned = (int64_t)host[sl::ST_SCANNED];
    out->steps = s->stat_steps;
    out->reconstructs = s->stat_steps;
  }
  s->stat_nodes = s->stat_steps = 0;
  if (aborted) return SL_EHIP;
  if (host[sl::ST_SEARCH_FAIL]) return SL_ESEARCH;
  if (host[sl::ST_NEWTON_FAIL]) return SL_ENEWTON;
  if (host[sl::ST_NONFINITE]) return SL_ENONFINITE;
  return SL_OK;
}

int sl_server_info(const sl_server* s, sl_server_status* out) {
  if (!s || !out) return SL_EINVAL;
  out->active = (int)s->active.size();
  out->finished = (int)s->finished.size();
  out->bytes_in_use = s->in_use;
  out->bytes_free = 0;
  for (const auto& kv : s->free_blocks) out->bytes_free += kv.second;
  out->ticks = s->tick;
  out->completed_ticks = s->completed_tick;
  return SL_OK;
}

}  // extern "C"
