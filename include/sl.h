/*
 * sl.h - C ABI of the MI355X (gfx950) forward semi-Lagrangian advection library.
 *
 * The library advects N scalar fields by a prescribed velocity on a regular,
 * periodic, node-centred reference grid in 2-D or 3-D, following the scheme of
 * Becerra-Sagredo, Malaga & Mandujano ("Moments Preserving and high-resolution
 * Semi-Lagrangian Advection Scheme"):
 *
 *   sl_step        integrates the trajectories of the material-lattice nodes
 *                  over one time step (Sec. 2, eqs. "momento" and "vel": the
 *                  lattice starts on the reference grid and moves with the
 *                  flow; fourth-order Runge-Kutta or the low-storage
 *                  third-order scheme of Williamson the paper cites);
 *   sl_reconstruct reconstructs every field on the reference grid from the
 *                  moved lattice (Sec. 2.1-2.3): per mesh node it finds the
 *                  deformed host element, inverts the multilinear (Z0) element
 *                  map with Newton's method (eq. "mapping1"), lowers the
 *                  Z-spline order while a point flagged by the jump criterion
 *                  lies in the stencil, and evaluates the tensor-product
 *                  cardinal Z-spline sum (eq. "multiZ", Appendix).  The
 *                  lattice is then reset onto the grid.
 *
 * Conventions
 *   - Grid: n[a] nodes along axis a (a = 0 is x), spacing h_a = length[a]/n[a],
 *     node positions x_i = i*h; every axis is periodic.
 *   - Field arrays: one device array per field, n[0]*n[1](*n[2]) elements of
 *     the value precision, x fastest (C order [z][y][x]).
 *   - Lattice displacements: kept in the caller's workspace in FP64, in cell
 *     units, structure-of-arrays; positions are never wrapped.
 *   - Value precision SL_FP64: everything in FP64.  SL_FP32: field values,
 *     Z-spline weights and sums in FP32; trajectories, the element search and
 *     the Newton inversion in FP64; jump flags evaluated in FP64 from the
 *     stored values.
 *
 * Ownership and errors
 *   - The caller owns all device memory (fields and workspace) and streams.
 *     The library never allocates device memory; it keeps only host-side
 *     descriptors.  Device pointers must stay valid until the work queued on
 *     the stream has completed (e.g. until sl_sync returns).
 *   - Every call returns SL_OK (0) or a negative sl_status.  Launch calls are
 *     asynchronous on the given HIP stream (NULL = the null stream); errors
 *     found on the device (search or Newton failure, non-finite output) are
 *     counted in the workspace and reported by sl_sync.  No call aborts or
 *     throws across the ABI.
 *   - A grid handle may be used from one host thread at a time.
 */
#ifndef SL_H
#define SL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SL_MAX_DIM 3
#define SL_MAX_FIELDS 8
#define SL_MAX_MODES 32
#define SL_VERSION 100

typedef enum sl_status {
  SL_OK = 0,
  SL_EINVAL = -1,      /* invalid argument or descriptor */
  SL_ENOMEM = -2,      /* host allocation failed */
  SL_EHIP = -3,        /* a HIP runtime call failed */
  SL_ESEARCH = -4,     /* a mesh node's host element was not found */
  SL_ENEWTON = -5,     /* Newton did not converge in the host element */
  SL_ENONFINITE = -6,  /* a reconstructed value is NaN or infinite */
  SL_EBUSY = -7,       /* no room (serving: HBM budget or slots exhausted) */
  SL_ESTATE = -8,      /* call out of order (e.g. reconstruct before step) */
  SL_ENOTFOUND = -9,   /* unknown request id */
  SL_ETOOBIG = -10     /* the grid needs more than the static scratch holds */
} sl_status;

enum { SL_FP64 = 0, SL_FP32 = 1 };
enum { SL_RK4 = 0, SL_RK3_WILLIAMSON = 1 };

/* Prescribed velocity families, in physical coordinates (x, y, z):
 *   SL_VEL_UNIFORM     u = (p0, p1, p2)
 *   SL_VEL_SOLID_BODY  u = p0 * (-(y - p2), x - p1, 0): rotation about (p1, p2)
 *   SL_VEL_SWIRL2D     u =  p1 sin^2(pi x) sin(2 pi y) cos(pi t / p0)
 *                      v = -p1 sin^2(pi y) sin(2 pi x) cos(pi t / p0)
 *   SL_VEL_DEFORM3D    u =  2 p1 sin^2(pi x) sin(2 pi y) sin(2 pi z) c
 *                      v =   -p1 sin(2 pi x) sin^2(pi y) sin(2 pi z) c
 *                      w =   -p1 sin(2 pi x) sin(2 pi y) sin^2(pi z) c,
 *                      c = cos(pi t / p0)
 *   SL_VEL_FOURIER     divergence-free sum of nmodes modes; mode q is the row
 *                      modes[7q .. 7q+6] = (k_x, k_y, k_z, a_x, a_y, a_z, phase)
 *                      with integer wave vector k, theta = 2 pi sum_a k_a x_a /
 *                      length[a] + phase and |k|^2 = sum_a k_a^2:
 *                      2-D: psi = sum a_x / |k|^2 sin(theta), u = (psi_y, -psi_x)
 *                      3-D: A = sum a / |k|^2 sin(theta),     u = curl A
 *                      all multiplied by p0.
 *   SL_VEL_GRIDDED     u given on the mesh nodes (sl_set_velocity_field) and
 *                      interpolated at the trajectory points with the
 *                      tensor-product cardinal Z-spline of order p0 = 0, 1 or
 *                      2 (eq. "multiZ" applied to the samples; periodic).  The
 *                      paper lets the velocity be given or carried with the
 *                      fields (Sec. 2); the samples are held fixed within a
 *                      step (all stages of a step use them).
 *   SL_VEL_CARRIED     u is transported with the fields: fields 0..dim-1 hold
 *                      its components.  With no right-hand side (Burgers'
 *                      equation Du/Dt = 0, Sec. 3) each lattice node keeps the
 *                      velocity it had at the last reset and moves on a
 *                      straight line.  Runs through sl_advance (which holds
 *                      the fields); needs nfields >= dim.                     */
enum {
  SL_VEL_UNIFORM = 0,
  SL_VEL_SOLID_BODY = 1,
  SL_VEL_SWIRL2D = 2,
  SL_VEL_DEFORM3D = 3,
  SL_VEL_FOURIER = 4,
  SL_VEL_GRIDDED = 5,
  SL_VEL_CARRIED = 6
};

/* Source terms, the right-hand side S_i of the transport equations (Sec. 2,
 * eq. "momento"), with spatial derivatives taken by centred finite differences
 * on the reference mesh (2m+1 points for the Z-spline order m in use, at least
 * three: the rules whose values the Z-splines' derivatives take at the knots,
 * eq. "matchder"):
 *   SL_SRC_NONE           pure transport
 *   SL_SRC_SHALLOW_WATER  the 2-D shallow-water system of eq. "nlsw" with
 *                         fields (u1, u2, h, passive ...), a carried velocity
 *                         and source_p = (fc, beta, y0, nu):
 *                           S_h  = -(1 + h) div u
 *                           S_u  = -grad h - f u_perp + nu div[(1 + h)(grad u +
 *                                  grad u^T)],  u_perp = (-u2, u1),
 *                           f    = fc + beta (y - y0)
 *                         (the paper's equatorial beta plane is fc = 0, beta =
 *                         f0, y0 the equator).  Needs dim 2, SL_VEL_CARRIED,
 *                         nfields >= 3, SL_RK3_WILLIAMSON and
 *                         reconstruct_every 1; runs through sl_advance only.
 *   A step integrates every lattice node's position and values with the
 *   low-storage RK3 of Williamson: each stage takes the stage fields on the
 *   mesh (the fields at t, then the reconstruction of the lattice's stage
 *   values), evaluates S there, and advances each node with its own velocity
 *   and S interpolated at its position with the order-m Z-spline; the fields
 *   at t + dt are the reconstruction of the final lattice values (three
 *   reconstructions per step). */
enum { SL_SRC_NONE = 0, SL_SRC_SHALLOW_WATER = 1 };

typedef struct sl_velocity {
  int kind;
  double p[8];
  int nmodes;            /* SL_VEL_FOURIER: 1..SL_MAX_MODES */
  const double *modes;   /* host memory, nmodes x 7 doubles; copied at create */
} sl_velocity;

typedef struct sl_grid_desc {
  int dim;                /* 2 or 3 */
  int64_t n[3];           /* nodes per axis, x first: 6 <= n[a] <= 2^24 (the quintic
                           * stencil fits the periodic grid once), n[1] <= 262140 and
                           * n[2] <= 65535 (launch-grid limits), fewer than 2^30
                           * nodes in all (SL_EINVAL otherwise) */
  double length[3];       /* physical extent per axis, > 0 */
  int nfields;            /* 1..SL_MAX_FIELDS */
  int value_prec;         /* SL_FP64 or SL_FP32 */
  int order_max;          /* highest Z-spline order m: 0 (linear), 1, 2 */
  int limiter;            /* 1: jump criterion of Sec. 2.3 lowers the order */
  double limiter_theta;   /* jump threshold, 0.25 in the paper */
  int integrator;         /* SL_RK4 or SL_RK3_WILLIAMSON */
  int reconstruct_every;  /* lattice steps between reconstructions, >= 1 */
  sl_velocity vel;
  int newton_max_iter;    /* Newton iterations per element, 20 */
  double newton_tol;      /* stop when max |delta xi| <= tol (cells), 1e-14 */
  int walk_max;           /* element-walk moves before the fallback scan, 32 */
  int scan_radius;        /* half-width of the fallback scan box, 4 */
  double eps_inside;      /* slack on the unit cube when accepting, 1e-12 */
  int source;             /* SL_SRC_NONE or SL_SRC_SHALLOW_WATER */
  double source_p[4];     /* source parameters, see SL_SRC_SHALLOW_WATER */
  int64_t offset[3];      /* index of node 0 in a larger periodic lattice (a shard of
                           * it; x first, default 0): trajectories are integrated at
                           * x_i = (i + offset) * h, so a shard's lattice moves exactly
                           * as the same nodes of the whole grid.  Its field arrays
                           * still wrap at n[a]: only nodes whose stencils stay clear
                           * of the shard's edges (a halo of at least the largest
                           * displacement plus 4 nodes) match the whole grid.  Not
                           * with SL_VEL_GRIDDED or a source term; |offset| < 2^30. */
  int limiter_pass;       /* where a 2-D grid evaluates the jump flags (Sec. 2.3):
                           * SL_LIMITER_AUTO (default: inside the reconstruction
                           * tiles below 2^22 nodes, a separate order-word pass
                           * from there up), SL_LIMITER_IN_TILES or
                           * SL_LIMITER_ORDER_WORDS.  Both give the same orders
                           * and results; 3-D grids always take the separate
                           * pass. */
} sl_grid_desc;

enum { SL_LIMITER_AUTO = 0, SL_LIMITER_IN_TILES = 1, SL_LIMITER_ORDER_WORDS = 2 };

/* Counters accumulated on the device since the last sl_sync. */
typedef struct sl_stats {
  int64_t nodes;           /* mesh-node reconstructions */
  int64_t search_fail;     /* nodes whose host element was not found */
  int64_t newton_fail;     /* nodes whose Newton solve did not converge */
  int64_t nonfinite;       /* field values reconstructed as NaN/Inf */
  int64_t order_hist[3];   /* field-node reconstructions per order used */
  int64_t walked;          /* nodes whose search left the start cell */
  int64_t scanned;         /* nodes located by the fallback scan */
  int64_t steps;           /* trajectory steps launched */
  int64_t reconstructs;    /* reconstructions launched */
} sl_stats;

typedef struct sl_grid sl_grid;

/* Fill a descriptor with the defaults listed above (2-D, FP64, Z2, limiter
 * off, theta 0.25, RK4, K = 1, zero uniform velocity, unit lengths). */
void sl_grid_desc_init(sl_grid_desc *desc);

/* Validate a descriptor and create a grid handle (host only, no device work).
 * Errors: SL_EINVAL (bad descriptor or NULL), SL_ENOMEM. */
int sl_create_grid(const sl_grid_desc *desc, sl_grid **out);

/* Destroy a handle; NULL is accepted. */
int sl_destroy_grid(sl_grid *grid);

/* Device bytes the caller must provide as `workspace` to the calls below
 * (lattice displacements, device counters, limiter order words and, for the
 * periodic velocity families, a per-axis sin/cos table that sl_advance fills
 * at each call); 0 for a NULL handle. The workspace must be 256-byte aligned
 * and zero-filled before its first use. */
size_t sl_workspace_bytes(const sl_grid *grid);

/* SL_VEL_GRIDDED: the velocity samples for later sl_step / sl_advance calls.
 * `components` holds `dim` device pointers (x first), each n[0]*n[1](*n[2])
 * FP64 values in physical units on the mesh nodes, x fastest.  The caller
 * owns them; they must stay valid until the launches that use them have run
 * (each launch reads the pointers current when it is queued).
 * Errors: SL_EINVAL (NULL argument, or the grid's velocity is not gridded). */
int sl_set_velocity_field(sl_grid *grid, const double *const *components);

/* Integrate the lattice trajectories over [t, t+dt] (Sec. 2).  The first step
 * after a reset starts every lattice node on its mesh node; later steps
 * continue from the stored displacement.  Asynchronous on `stream`.
 * Errors: SL_EINVAL (also for a carried velocity, which needs the fields:
 * use sl_advance), SL_ESTATE (gridded velocity without samples), SL_EHIP. */
int sl_step(sl_grid *grid, void *workspace, double t, double dt, void *stream);

/* Reconstruct all fields on the mesh from the moved lattice and reset the
 * lattice (Sec. 2.1-2.3).  fields_in / fields_out are host arrays of nfields
 * device pointers to caller-owned arrays in the grid's value precision; an
 * output array must not alias any input array.  Asynchronous on `stream`.
 * Errors: SL_EINVAL, SL_ESTATE (no sl_step since the last reset), SL_EHIP. */
int sl_reconstruct(sl_grid *grid, void *workspace, const void *const *fields_in,
                   void *const *fields_out, void *stream);

/* Wait for `stream`, copy the device counters into *stats (may be NULL) and
 * clear them.  Returns the first device-side error class seen since the last
 * sync (SL_ESEARCH, SL_ENEWTON, SL_ENONFINITE, in that priority), else SL_OK,
 * or SL_EHIP / SL_EINVAL. */
int sl_sync(sl_grid *grid, void *workspace, void *stream, sl_stats *stats);

/* Run nsteps steps from t0 with a constant dt: every reconstruct_every steps
 * the lattice is reconstructed onto the mesh and reset.  The fields ping-pong
 * between the caller-owned sets fields_a (initial values) and fields_b;
 * *result_in_b (may be NULL) tells which set holds the result.  nsteps must be
 * a multiple of reconstruct_every and the lattice must be reset (no pending
 * sl_step).  Asynchronous on `stream`; equivalent to the sequence of sl_step /
 * sl_reconstruct calls but without per-call host overhead.  With a source term
 * it is the only way to step (see SL_SRC_SHALLOW_WATER).
 * Errors: SL_EINVAL, SL_ESTATE, SL_EHIP. */
int sl_advance(sl_grid *grid, void *workspace, void *const *fields_a,
               void *const *fields_b, double t0, double dt, int nsteps,
               void *stream, int *result_in_b);

/* sl_advance without a workspace argument, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  The lattice displacements, limiter words and device
 * counters live in a scratch array of SL_STATIC_SCRATCH_BYTES that the
 * library holds on each device it runs on until the process ends; the call
 * allocates nothing, host or device (the caller still owns the two field
 * sets, the stream and `counters`).
 *   - Runs on the current device; `stream` must belong to it.
 *   - Same arguments, semantics, kernels and results as sl_advance.
 *   - The scratch's counters are cleared at the start of each call (by a fill
 *     kernel on `stream`).  counters (device memory, may be NULL) receives
 *     SL_STATIC_COUNTERS int64 values once the call's kernels have run:
 *     search failures, Newton failures, non-finite values, field-node
 *     reconstructions at order 0 and at order 1, walked nodes, scanned nodes,
 *     and 0.  The grid's own counters (sl_sync) are not touched.
 *   - Every call on one device shares that device's scratch and leaves its
 *     contents there: calls that overlap on one device (on different streams,
 *     or from different host threads) race and must be serialised by the
 *     caller.
 * Errors: SL_ETOOBIG when sl_workspace_bytes(grid) exceeds
 * SL_STATIC_SCRATCH_BYTES, SL_EHIP, and those of sl_advance. */
#define SL_STATIC_SCRATCH_BYTES ((size_t)128 << 20)
#define SL_STATIC_COUNTERS 8
int sl_advance_static(sl_grid *grid, void *const *fields_a, void *const *fields_b,
                      double t0, double dt, int nsteps, void *stream, int *result_in_b,
                      int64_t *counters);

/* Kernel timing: when enabled, the timed launches of the grid carry HIP
 * events in their dispatch packets.  Kinds: trajectories (sl_step), the
 * reconstruction kernel, the limiter order-word kernels that precede it in
 * sl_reconstruct (none when the limiter is off), and the source-term kernels
 * (SL_SRC_SHALLOW_WATER). */
typedef struct sl_profile {
  int64_t traj_launches;
  double traj_ms;          /* summed kernel time of the timed trajectory launches */
  int64_t recon_launches;
  double recon_ms;         /* summed kernel time of the timed reconstruction launches */
  int64_t orders_launches;
  double orders_ms;        /* first order-word kernel start to last one's end, summed */
  int64_t source_launches;
  double source_ms;        /* source-term kernels (mesh right-hand side, lattice stage) */
} sl_profile;

/* Time every `period`-th launch of each kind from now on (1: every launch;
 * 0 or less: off).  Events add a few microseconds between kernels, so a
 * period above 1 keeps a long run close to its untimed speed. */
int sl_profile_enable(sl_grid *grid, int period);

/* Wait for the timed launches, report their totals and clear them. */
int sl_profile_read(sl_grid *grid, sl_profile *out);

/* Device pointer to the lattice displacement along `axis` (0 = x) inside
 * `workspace`: n[0]*n[1](*n[2]) doubles in cell units, x fastest, valid after
 * sl_step and until the next sl_step after a reconstruction.  NULL on a bad
 * argument. */
const double *sl_displacement(const sl_grid *grid, const void *workspace, int axis);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of many independent 2-D problems.
 *
 * The caller provides one device arena; its size is the HBM budget.  Each
 * admitted request receives its own field buffers and lattice workspace from
 * the arena (or SL_EBUSY when they do not fit or max_requests are active).
 * Every sl_server_tick advances each active request by one step
 * (trajectories, then reconstruction and lattice reset, as sl_step +
 * sl_reconstruct with reconstruct_every = 1) through batched launches on the
 * server's stream; requests join between ticks and leave when their step
 * count is reached.  A request's result is bitwise the same as running it
 * alone through sl_advance.  2-D grids only; all velocity families but
 * SL_VEL_DEFORM3D.  A server is used from one host thread at a time.
 * ------------------------------------------------------------------------ */
typedef struct sl_server sl_server;

typedef struct sl_server_status {
  int active;              /* requests still stepping */
  int finished;            /* requests done stepping, not yet fetched */
  size_t bytes_in_use;     /* arena bytes held by requests */
  size_t bytes_free;       /* arena bytes available to admissions */
  int64_t ticks;           /* ticks enqueued */
  int64_t completed_ticks; /* ticks known to have finished on the device */
} sl_server_status;

/* Arena bytes the server keeps for itself (request table, counters, the
 * window kernels' queues) with room for max_requests requests (0 if
 * invalid); the rest of the arena holds the requests. */
size_t sl_server_arena_overhead(int max_requests);

/* Arena bytes one request with this descriptor occupies (0 if invalid). */
size_t sl_server_request_bytes(const sl_grid_desc *desc);

/* Create a server over the device arena [arena, arena + arena_bytes)
 * (256-byte aligned, caller-owned, must outlive the server).  At most
 * max_requests requests are resident; sl_server_tick blocks the host while
 * more than max_inflight ticks are queued on `stream`.  Errors: SL_EINVAL,
 * SL_ENOMEM, SL_EHIP. */
int sl_server_create(void *arena, size_t arena_bytes, int max_requests,
                     int max_inflight, void *stream, sl_server **out);

/* Wait for the stream and destroy the server (NULL accepted). */
int sl_server_destroy(sl_server *server);

/* Admit a request: copy its initial fields (device pointers in the grid's
 * value precision; the copy is queued on the server's stream, so the sources
 * must stay valid until that stream reaches it) into the arena and schedule
 * nsteps steps of dt from t0.  *id identifies it.
 * Errors: SL_EINVAL (bad descriptor, 3-D grid, gridded or carried velocity,
 * reconstruct_every != 1),
 * SL_EBUSY (no room), SL_EHIP. */
int sl_server_admit(sl_server *server, const sl_grid_desc *desc,
                    const void *const *fields_in, double t0, double dt, int nsteps,
                    int64_t *id);

/* Advance every active request by one step (up to `window` steps in
 * SL_SERVE_QUEUED mode, see sl_server_set_mode); *active (may be NULL)
 * receives the number still stepping afterwards.  Errors: SL_EINVAL, SL_EHIP. */
int sl_server_tick(sl_server *server, int *active);

/* Report up to max_ids requests whose last step has completed on the device
 * and that were not reported before.  Never blocks. */
int sl_server_poll(sl_server *server, int64_t *done_ids, int max_ids, int *ndone);

/* Copy a finished request's fields into caller buffers (asynchronous on the
 * server's stream) and release its arena memory.  SL_ENOTFOUND for an unknown
 * or unfinished id. */
int sl_server_fetch(sl_server *server, int64_t id, void *const *fields_out);

/* Wait for the stream; report and clear the counters accumulated by all
 * requests since the last call (nodes and steps count request steps; status
 * as for sl_sync, and SL_EHIP if a queued launch gave up waiting). */
int sl_server_sync(sl_server *server, sl_stats *stats);

/* How sl_server_tick launches the work of a tick.
 *   SL_SERVE_BATCHED  one batched reconstruction launch per value precision
 *                     and field count, every request one step per tick
 *                     (window must be 1).  The default.
 *   SL_SERVE_QUEUED   one launch per value precision and field count runs
 *                     `window` (1..16) steps of every request of the group:
 *                     the tiles of all those steps sit in device-side queues
 *                     (one per XCD, in step order), each workgroup takes the
 *                     next tile of the queue of the XCD it runs on, and a
 *                     request's step starts once every tile of its previous
 *                     step is done (device-side counts, no host round trip).
 *                     Requests with more than 4 fields keep batched
 *                     launches, one step per tick.
 * Results are bitwise the same in both modes.  Errors: SL_EINVAL. */
enum { SL_SERVE_BATCHED = 0, SL_SERVE_QUEUED = 1 };
int sl_server_set_mode(sl_server *server, int mode, int window);

/* Occupancy of the server. */
int sl_server_info(const sl_server *server, sl_server_status *out);

/* Static text for a status code. */
const char *sl_strerror(int code);

/* Text of the last HIP runtime error this thread saw inside the library
 * (empty if none); the pointer stays valid for the thread's lifetime. */
const char *sl_error_detail(void);

/* SL_VERSION of the built library. */
int sl_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SL_H */
