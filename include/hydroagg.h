/*
 * hydroagg.h -- C ABI of libhydroagg.so: the aggregated FP64 sub-grid hydro
 * step on MI355X (gfx950).
 *
 * Operation.  One forward-Euler stage of the ideal-gas Euler equations on a
 * batch of independent octree sub-grids (the paper's Section IV-B "Hydro
 * Solver": piecewise-parabolic reconstruction, central-upwind fluxes at the
 * cell-face centres, flux-divergence update; Section V-A: an N^3 sub-grid
 * stored with a 3-cell ghost layer, (N+6)^3 cells per field).  The batch is
 * executed by ONE aggregated kernel launch per sub-grid shape class instead
 * of one launch per sub-grid (the paper's strategy 3, Section V-D).  gamma is
 * fixed at 5/3.
 *
 * Memory layout of one sub-grid (u_in, and u_out by default): float64,
 * structure of arrays [nfields][M][M][M], M = n + 6, x fastest, linear index
 * ((f*M + z)*M + y)*M + x.  Interior cells are x, y, z in [3, n+3).
 * With out_layout = HYDRO_OUT_INTERIOR, u_out holds the interior only:
 * [nfields][n][n][n], linear index ((f*n + z)*n + y)*n + x for interior cell
 * (x+3, y+3, z+3) of the stored layout -- every element is written, rows are
 * whole 64-byte multiples, and the buffer is (n/(n+6))^3 of the stored size.
 * Fields: 0 rho, 1 sx, 2 sy, 3 sz, 4 egas (total energy density), 5 tau
 * (passive entropy tracer), 6..10 partial densities of 5 species (nfields 11).
 *
 * Ownership.  All data pointers are DEVICE pointers owned by the caller; the
 * library never frees them and never keeps them past the completion of the
 * work that names them.  The library owns its descriptor tables, pinned
 * staging, events and streams, all created at initialisation / create time;
 * no device allocation happens on the step path.
 *
 * Asynchrony.  Calls only enqueue work.  Results are valid once the stream
 * (hydro_step) or the ticket (aggregator) has completed.  The caller keeps
 * every buffer alive until then.
 *
 * Errors.  Every call returns 0 on success or a negative code below; the
 * message of the last failure on the calling thread is hydro_last_error().
 */
#ifndef HYDROAGG_H
#define HYDROAGG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HYDRO_OK 0
#define HYDRO_EINVAL (-1)  /* bad argument (see each call)                   */
#define HYDRO_EHIP (-2)    /* a HIP runtime call failed; text in last_error  */
#define HYDRO_ENOMEM (-3)  /* no descriptor / slab space left                */
#define HYDRO_EAGAIN (-4)  /* admission refused (HBM budget); retry later    */

#define HYDRO_GHOST 3

/* Layouts of u_out (hydro_subgrid_t.out_layout). */
#define HYDRO_OUT_STORED 0    /* the (n+6)^3 layout of u_in; interior written */
#define HYDRO_OUT_INTERIOR 1  /* interior only, [nfields][n][n][n]            */

/* One sub-grid task: 32 bytes. */
typedef struct {
  const double *u_in; /* device; [nfields][M][M][M]; read-only                 */
  double *u_out;      /* device; layout per out_layout: the shape of u_in with
                         only the interior n^3 written (STORED), or the
                         interior alone (INTERIOR); must not overlap u_in     */
  int32_t n;          /* interior edge: 8, 12 or 16                            */
  int32_t nfields;    /* 6 or 11                                               */
  int32_t level;      /* octree level: cell width dx_s = dx * 2^-level, 0..30  */
  int32_t out_layout; /* HYDRO_OUT_STORED (0) or HYDRO_OUT_INTERIOR (1)       */
} hydro_subgrid_t;

/*
 * hydro_set_tile / hydro_get_tile -- the block ("tile") a sub-grid of class
 * (n, nfields) is stepped as: tile 8 = 8^3 blocks (one per 8^3 sub-grid, 8
 * per 16^3, 8 overlapping ones per 12^3), tile 4 = disjoint 4^3 blocks, four
 * per work-group.  Both compute every face from the same cells, so results
 * agree to rounding (the two kernels may contract the same expressions
 * differently); for a fixed tile they are bitwise reproducible and
 * independent of the batch.  The choice is made by the autotuner
 * (paper_2210_06438_amd/tune.py).  Defaults:
 * 8 for n = 8 and 16, 4 for n = 12.  Process-wide; read at every launch; a
 * plan re-captures its graph after a change.  Errors: HYDRO_EINVAL for an
 * unsupported class, a tile other than 4 or 8, or tile == NULL.
 */
int hydro_set_tile(int32_t n, int32_t nfields, int32_t tile);
int hydro_get_tile(int32_t n, int32_t nfields, int32_t *tile);

/*
 * hydro_step -- one stage for `count` sub-grids (paper Section IV-B), as one
 * aggregated launch per (n, nfields) class present in the batch; a batch of
 * several classes of one field count is ONE launch in which the classes run
 * side by side (results bitwise those of the per-class launches).
 *   sg       host array of `count` descriptors (copied before return).
 *   dt       time-step, >= 0 and finite.  dt = 0 leaves the interior equal to
 *            u_in and still produces amax (used to pick the Courant dt).
 *   dx       cell width at level 0, > 0 and finite.
 *   amax_dev device array of `count` doubles or NULL: amax_dev[s] = max over
 *            all 3(n+1)n^2 faces of sub-grid s of max(a+, -a-), the largest
 *            signal speed (the quantity behind the Courant limit, Sec. IV-B).
 *   stream   hipStream_t to enqueue on (NULL = default stream).
 * Per sub-grid: U_out = U - dt/dx_s * sum_d (F_{d,i+1/2} - F_{d,i-1/2}) on
 * the interior; in the stored layout the ghost cells of u_out are never
 * written.  Both layouts give bitwise the same values.
 * Errors: HYDRO_EINVAL for sg == NULL with count > 0, count < 0, n not in
 * {8,12,16}, nfields not in {6,11}, level outside 0..30, out_layout not 0 or
 * 1, NULL u_in/u_out, u_out overlapping u_in (per sub-grid), dt < 0 or not
 * finite, dx <= 0 or not finite;
 * HYDRO_EHIP if a launch or copy fails.  count = 0 is a no-op success.
 * Thread safety: any number of host threads may call hydro_step at once
 * (each on its own stream or the same one); the library's descriptor
 * staging slots are taken in turn and each is held until its copy and
 * launches are enqueued, and reused only after that work has completed.
 */
int hydro_step(const hydro_subgrid_t *sg, int32_t count, double dt, double dx,
               double *amax_dev, void *stream);

/*
 * hydro_step_static -- hydro_step for callers that cannot allocate memory:
 * code that runs under stream capture, tight serving loops, and harnesses
 * that forbid allocation.  Same arguments, launches, results (bitwise) and
 * errors as hydro_step, but the call never allocates device or host memory,
 * at its first call or later: the descriptor table goes to a static device
 * array of HYDRO_STATIC_MAX descriptors (32 bytes each: 256 KiB, held by every
 * GPU the library runs on until the process ends) through a static host
 * staging array of the same size.  Errors as hydro_step, plus HYDRO_EINVAL
 * when count > HYDRO_STATIC_MAX.
 * Concurrency: every call on one GPU shares that GPU's arrays, which keep the
 * last call's descriptors.  Calls are serialised on the host, and calls on
 * one stream are ordered; calls whose work may overlap on one GPU (different
 * streams, or a graph that holds the call replayed beside another call) race
 * on the device table and give wrong results.
 */
#define HYDRO_STATIC_MAX 8192
int hydro_step_static(const hydro_subgrid_t *sg, int32_t count, double dt,
                      double dx, double *amax_dev, void *stream);

/*
 * hydro_step_streams -- the paper's strategy 2 (Section V-C, implicit work
 * aggregation): the same kernel launched once per sub-grid, the launches
 * dealt round-robin to n_streams (1..128) library-owned streams, so that
 * the GPU may run the small kernels side by side.  The pool streams start
 * after the work already queued on `stream` and `stream` continues after
 * all of them (an event each way), so the call is ordered on `stream` like
 * hydro_step.  The pool's streams are created at first use, up to the
 * largest n_streams asked for, and kept until the process ends; a call with
 * count = 0 only creates them (set-up).  Calls are serialised by a mutex per
 * device.  Results, amax and errors as hydro_step (results bitwise equal to
 * it); HYDRO_EINVAL for n_streams outside 1..128.
 */
int hydro_step_streams(const hydro_subgrid_t *sg, int32_t count, double dt,
                       double dx, double *amax_dev, int32_t n_streams,
                       void *stream);

/*
 * hydro_step26 -- the 26-point form of the aggregated step (Section IV-B):
 * the evolved variables are reconstructed (piecewise-parabolic, with the
 * monotonicity constraint) at the 26 points of each cell's surface -- face
 * centres, edge midpoints and vertices, each along the line of cells toward
 * that point -- central-upwind fluxes are evaluated at the 9 points of
 * every face, and Simpson's rule in both transverse directions integrates
 * them over the face (weights 16, 4, 1 over 36 for centre, edge midpoints,
 * vertices).  hydro_step evaluates the face centres only.  Sub-grids of
 * n = 8, all of one field count (HYDRO_EINVAL otherwise); their edge and
 * corner ghosts are read.  Arguments, layouts, amax (over all 9 points of
 * every face) and other errors as hydro_step.  One launch per call (of at
 * most 65536 sub-grids), one 576-lane work-group per sub-grid.
 */
int hydro_step26(const hydro_subgrid_t *sg, int32_t count, double dt,
                 double dx, double *amax_dev, void *stream);

/*
 * hydro_step_each -- the non-aggregated baseline: the same kernel launched
 * once per sub-grid (the paper's "1 executor, max aggregated 1" setting,
 * Section VI-B), every launch on `stream`, each carrying its one descriptor
 * in its kernel arguments.  Same arguments, results and errors as
 * hydro_step; results are bitwise identical to it.
 */
int hydro_step_each(const hydro_subgrid_t *sg, int32_t count, double dt,
                    double dx, double *amax_dev, void *stream);

/*
 * Plans: a fixed batch whose descriptor table is uploaded once, for callers
 * that step the same set of sub-grids repeatedly (every stage of a time-step
 * on device-resident state).  hydro_plan_create copies `sg` into a
 * plan-owned device table (this allocates, so it belongs to set-up, not to
 * the step path).  hydro_plan_step then only launches kernels, grouped as
 * in hydro_step, with its results and errors.
 * hydro_plan_launch_graph runs the same launches as ONE hipGraph launch on
 * `stream`, the classes of one field count as one launch; with two field
 * counts, classes of at least 1024 work-groups become independent branches
 * of the graph and run concurrently (results are those of
 * hydro_plan_step, bit for bit); the graph is captured on private streams
 * at first use and
 * captured again whenever dt, dx, amax_dev or a class's tile change.  A plan may be used
 * from one host thread at a time; hydro_plan_destroy waits for its work.
 */
typedef struct hydro_plan hydro_plan_t;
int hydro_plan_create(hydro_plan_t **out, const hydro_subgrid_t *sg,
                      int32_t count);
int hydro_plan_step(hydro_plan_t *plan, double dt, double dx,
                    double *amax_dev, void *stream);
int hydro_plan_launch_graph(hydro_plan_t *plan, double dt, double dx,
                            double *amax_dev, void *stream);
int hydro_plan_destroy(hydro_plan_t *plan);

/*
 * hydro_plan_pattern_floor -- a roofline reference, not a step: the HBM
 * access pattern of the aggregated 8^3 step without its arithmetic, over a
 * plan's batch (all sub-grids with n = 8 and one field count).  One launch
 * on `stream` reads exactly the cells the step reads, in the step's order
 * and lane roles, and writes each interior once in its descriptor's output
 * layout; the values written are the input interior plus a negligible
 * multiple of the ghost cells read (no physical meaning: u_out holds no step
 * result afterwards).  same_lds != 0 reserves the step kernel's LDS, so it
 * runs at the step's work-groups per CU; 0 lets as many run as registers
 * allow.  Its duration is what the step's data movement alone costs
 * (bench.py reports it beside the step's).
 * Errors: HYDRO_EINVAL for a NULL plan or a plan with another shape or two
 * field counts; HYDRO_EHIP if the launch fails.
 */
int hydro_plan_pattern_floor(hydro_plan_t *plan, int32_t same_lds,
                             void *stream);

/*
 * Bricks: a regular block of nb[0] x nb[1] x nb[2] sub-grids of one shape
 * (edge n, nfields fields, one octree level) tiling a rectangular domain of
 * n*nb[0] x n*nb[1] x n*nb[2] cells, each sub-grid stored as in hydro_step
 * ([nfields][M][M][M], M = n + 6) and the sub-grids contiguous in the order
 * s = (bz*nb[1] + by)*nb[0] + bx (x fastest).  A brick buffer holds
 * nb[0]*nb[1]*nb[2]*nfields*M^3 doubles.  bc[d] is the boundary condition of
 * the domain along axis d (x, y, z): HYDRO_BC_PERIODIC wraps around,
 * HYDRO_BC_OUTFLOW continues the domain by its outermost cell (zero
 * gradient).  This is the multi-sub-grid state of the paper's time-step,
 * whose three solver iterations (Section VI-A) each read ghost layers that
 * the neighbouring sub-grids' interiors fill (Section V-A: sub-grids with
 * 3-cell ghost layers).
 */
#define HYDRO_BC_PERIODIC 0
#define HYDRO_BC_OUTFLOW 1

typedef struct {
  int32_t n;       /* 8, 12 or 16                                     */
  int32_t nfields; /* 6 or 11                                         */
  int32_t nb[3];   /* sub-grids along x, y, z, each >= 1              */
  int32_t bc[3];   /* HYDRO_BC_PERIODIC or HYDRO_BC_OUTFLOW per axis  */
  int32_t level;   /* octree level of every sub-grid, 0..30           */
} hydro_brick_t;

/*
 * hydro_ghost_fill -- set every ghost cell (faces, edges and corners) of
 * every sub-grid of the brick buffer u, in place, to the value of the domain
 * cell it stands for: the interior cell of the neighbouring sub-grid, or,
 * beyond the domain, the cell given by the boundary condition of each axis
 * applied independently.  Interior cells are only read.  Bitwise a copy.
 * Errors: HYDRO_EINVAL for a NULL brick or buffer, an unsupported shape, a
 * count below 1 or above 2^20 sub-grids, a bad bc or level, or a buffer not
 * 16-byte aligned; HYDRO_EHIP if the launch fails.  Enqueues on `stream`.
 */
int hydro_ghost_fill(const hydro_brick_t *brick, double *u, void *stream);

/*
 * hydro_ghost_fill_faces -- as hydro_ghost_fill, for the face ghosts only:
 * the six 3-deep slabs whose other two coordinates are interior, which are
 * the only ghost cells the face-centre step reads (it marches the lines
 * whose transverse coordinates are interior, Section IV-B).  Edge and corner
 * ghosts are left unchanged; call hydro_ghost_fill before a step that reads
 * them (hydro_step26).  Same arguments and errors as hydro_ghost_fill.
 */
int hydro_ghost_fill_faces(const hydro_brick_t *brick, double *u, void *stream);

/*
 * SSP-RK3 time-step on a device-resident brick: the paper's time-step of
 * three solver iterations (Section VI-A) composed from hydro_step as the
 * three-stage strong-stability-preserving Runge-Kutta method of Shu and
 * Osher (J. Comput. Phys. 77, 1988), with E(V) = one hydro_step stage of V:
 *   U1 = E(U0),  U2 = 3/4 U0 + 1/4 E(U1),  U3 = 1/3 U0 + 2/3 E(U2),
 * each combination rounded as a x + b y with the two products and the sum
 * rounded once (for n = 8 formed in the step's own stores),
 * each stage's result with its face ghosts refilled (the stage reads no edge
 * or corner ghost) before the next stage reads it: for n = 8 the stage
 * kernel writes every stored value near a face also into the face ghost it
 * stands for (bitwise what hydro_ghost_fill_faces would write), for n = 12
 * and 16 hydro_ghost_fill_faces follows the stage.
 * hydro_rk3_create binds the brick to three caller-owned device brick
 * buffers: u (the state, with face ghosts filled on entry; it holds U3,
 * face ghosts filled, after a step; its edge and corner ghosts are left as
 * they were) and two work buffers w and s (their contents are
 * overwritten).  It creates the stages' aggregated steps (E(u) into w, E(w)
 * into s, E(s) into u for n = 8 or into w otherwise) and their descriptor
 * tables, so it allocates and belongs to set-up.  The buffers must not
 * overlap and must stay alive until hydro_rk3_destroy.
 * hydro_rk3_stage(rk, k, ...) runs stage k = 1, 2 or 3 alone (after stage 1,
 * w holds U1; after stage 2, s holds U2; after stage 3, u holds U3; each
 * with face ghosts), so that
 * the three calls in order are one time-step; hydro_rk3_step runs all three
 * as launches, hydro_rk3_launch_graph as ONE hipGraph launch (captured at
 * first use and again when dt, dx or amax_dev change; results bitwise those
 * of hydro_rk3_step).  dt >= 0 and dx > 0 as in hydro_step; amax_dev (device,
 * one double per sub-grid, or NULL) receives the amax of stage 1, i.e. of
 * the state the step starts from (hydro_step's definition); the later stages
 * write no amax.  Per step: for n = 8, 3 stage kernels; for n = 12 and 16,
 * 3 aggregated steps, 2 stage combinations and 3 face-ghost fills.  A
 * time-step object may be used from one host thread at a
 * time; hydro_rk3_destroy waits for its work.
 * Errors: as hydro_step and hydro_ghost_fill; HYDRO_EINVAL for k outside
 * 1..3 or overlapping buffers.
 */
typedef struct hydro_rk3 hydro_rk3_t;
int hydro_rk3_create(hydro_rk3_t **out, const hydro_brick_t *brick, double *u,
                     double *w, double *s);
int hydro_rk3_stage(hydro_rk3_t *rk, int32_t k, double dt, double dx,
                    double *amax_dev, void *stream);
int hydro_rk3_step(hydro_rk3_t *rk, double dt, double dx, double *amax_dev,
                   void *stream);
int hydro_rk3_launch_graph(hydro_rk3_t *rk, double dt, double dx,
                           double *amax_dev, void *stream);
int hydro_rk3_destroy(hydro_rk3_t *rk);

/*
 * Aggregation regions: the paper's application-independent aggregation
 * executor (Section V-D).  A region is a piece of task code -- staging
 * buffers, filling them, copies, a kernel launch -- that several tasks (host
 * threads) may run together as one team, each on its own chunk of shared
 * buffers, the GPU work issued once for the whole team:
 *   hydro_region_enter   blocks until the task enters with a team: at once
 *                        (with whoever waits) when one of the region's
 *                        n_streams executors is idle, else when max_team
 *                        tasks wait (that full team enters anyway and queues
 *                        behind the team on an executor; two team slots per
 *                        executor), else when an executor frees.  *task
 *                        receives its team, index (0..size-1) and size.
 *   hydro_region_alloc   the k-th call of every member is one team buffer:
 *                        the first member reserves size x stride bytes
 *                        (stride = bytes rounded up to 8) of the team's
 *                        arena; each member gets its chunk (host mirror and
 *                        device address) at index x stride.  Every member
 *                        must ask for the same bytes.
 *   hydro_region_buffer  device base address and stride of a team buffer
 *                        (for kernel arguments).
 *   hydro_region_upload / _download  host mirror to device / back, of a
 *                        whole team buffer, once, when the last member calls.
 *   hydro_region_launch  `kernel` (a __global__ function of this library,
 *                        hydro_region_kernel(), or of the caller's code) runs
 *                        once, when the last member calls, with size x
 *                        blocks_per_task work-groups of `threads` lanes and
 *                        the last caller's `args` (hipLaunchKernel style: an
 *                        array of pointers to each argument); the kernel finds
 *                        its member from its work-group index.
 *   hydro_region_wait    the last member records the team's completion;
 *                        every member returns when the team's device work has
 *                        finished.  Its downloaded chunks are then valid until
 *                        it calls hydro_region_leave; only leave may follow.
 *   hydro_region_leave   as hydro_region_wait if the team has not recorded
 *                        its completion yet; when the last member has left,
 *                        the team's slot and arena may serve the next team
 *                        (read downloaded chunks between wait and leave).
 * Every member makes the same sequence of calls ("single GPU workload,
 * multiple tasks"); a call that differs from the team's (kind, bytes,
 * launch shape) fails the team with HYDRO_EINVAL, an arena overflow with
 * HYDRO_ENOMEM: every member's later calls return that error and nothing
 * more is issued for the team.  Every member must call leave exactly once
 * (that frees the team's slot).  hydro_region_create makes n_streams
 * (1..32) streams and 2 x n_streams arenas of arena_bytes device memory plus
 * pinned host mirrors; nothing is allocated afterwards.  Destroying a region
 * with tasks inside is undefined.
 */
typedef struct hydro_region hydro_region_t;
typedef struct {
  int32_t team;   /* team slot                         */
  int32_t index;  /* this member's index, 0..size-1    */
  int32_t size;   /* members of the team               */
  int32_t stream; /* the team's executor               */
  uint64_t id;    /* team serial number                */
} hydro_region_task_t;
typedef struct {
  uint64_t tasks, teams, full_teams, uploads, launches, downloads;
  uint64_t size_hist[11]; /* teams of size 1, 2-3, 4-7, ..., >= 1024 */
} hydro_region_stats_t;
int hydro_region_create(hydro_region_t **out, int32_t max_team,
                        int32_t n_streams, uint64_t arena_bytes);
int hydro_region_enter(hydro_region_t *r, hydro_region_task_t *task);
int hydro_region_alloc(hydro_region_t *r, const hydro_region_task_t *task,
                       uint64_t bytes, int32_t *buffer, void **host_chunk,
                       void **dev_chunk);
int hydro_region_buffer(hydro_region_t *r, const hydro_region_task_t *task,
                        int32_t buffer, void **dev_base, uint64_t *stride);
int hydro_region_upload(hydro_region_t *r, const hydro_region_task_t *task,
                        int32_t buffer);
int hydro_region_download(hydro_region_t *r, const hydro_region_task_t *task,
                          int32_t buffer);
int hydro_region_launch(hydro_region_t *r, const hydro_region_task_t *task,
                        const void *kernel, uint32_t blocks_per_task,
                        uint32_t threads, uint32_t shmem, void **args);
int hydro_region_wait(hydro_region_t *r, const hydro_region_task_t *task);
int hydro_region_leave(hydro_region_t *r, const hydro_region_task_t *task);
int hydro_region_stats(hydro_region_t *r, hydro_region_stats_t *out);
int hydro_region_destroy(hydro_region_t *r);

/*
 * Kernels of this library that run inside a region (NULL for another
 * value):
 *   HYDRO_REGION_STEP8_F6 / _F11: the aggregated 8^3 step, arguments
 *     (const hydro_subgrid_t *table, int32_t count, double dt, double dx,
 *      double *amax): member s's descriptor at table[s] (a team buffer of
 *     32-byte chunks), results as hydro_step, amax of member s at amax[s];
 *     blocks_per_task 1, threads 192.
 *   HYDRO_REGION_AXPBY: out = a x + b y over n doubles per member (the
 *     stage combination of a Runge-Kutta step), arguments
 *     (const hydro_region_axpby_t *table, int32_t count,
 *      int32_t blocks_per_task); threads 256.
 */
#define HYDRO_REGION_STEP8_F6 0
#define HYDRO_REGION_STEP8_F11 1
#define HYDRO_REGION_AXPBY 2
typedef struct {
  const double *x;
  const double *y;
  double *out;
  double a;
  double b;
  int64_t n;
} hydro_region_axpby_t;
const void *hydro_region_kernel(int32_t which);

/*
 * hydro_region_drive -- many independent host tasks through a region, as
 * the paper's tasks reach their kernel (Section V-D), for measurement:
 * n_threads host threads (1..256, created and joined by the call) take the
 * count tasks sg[0..count) in turn (count 1..2^20, every descriptor n = 8
 * with one field count, 6 or 11).
 *   mode HYDRO_DRIVE_REGION: each task enters region r, allocates a
 *     descriptor chunk and an amax chunk, copies its descriptor, uploads,
 *     launches the library's 8^3 step for the team, downloads, waits, reads
 *     its amax and leaves: one upload, launch and download per team.
 *   mode HYDRO_DRIVE_EACH: each task is one hydro_step launch of its own
 *     sub-grid on its thread's stream, then a wait for its amax (the
 *     non-aggregated baseline; r is not used and may be NULL).
 * Every sub-grid is stepped exactly as hydro_step steps it (bitwise).
 * amax_host (host, count doubles, or NULL) receives each task's amax;
 * *seconds the wall time from the moment every thread has made its set-up
 * (EACH: its stream and buffers) to the last join.
 * Errors: HYDRO_EINVAL for bad arguments; the first failing task's error
 * otherwise (the other threads then stop taking tasks).  Allocates (threads,
 * per-thread streams): set-up and measurement, not a step path.
 */
#define HYDRO_DRIVE_REGION 0
#define HYDRO_DRIVE_EACH 1
int hydro_region_drive(hydro_region_t *r, const hydro_subgrid_t *sg, int32_t count,
                       int32_t n_threads, double dt, double dx, int32_t mode,
                       double *amax_host, double *seconds);

/*
 * Aggregator: explicit work aggregation of fine-grained sub-grid tasks (the
 * paper's strategy 3, Section V-D).  Tasks submitted while the aggregator's
 * streams are busy are held and launched together as one batch (one kernel
 * per shape class) when the batch reaches max_width (the paper's "max
 * aggregated kernels"; 1 disables aggregation), when a stream is idle (if
 * flush_when_idle), when the oldest held task is timeout_us old (< 0: never),
 * on hydro_flush, or when a task with a different (dt, dx) arrives.
 * Admission is bounded: held plus in-flight tasks may not own more than
 * hbm_budget_bytes of output (0 = unbounded); hydro_submit then returns
 * HYDRO_EAGAIN and the caller retries after hydro_progress / completions.
 * n_streams (1..128) streams and all batch buffers are created by
 * hydro_agg_create; submit/flush/progress/poll never allocate.  Calls on one
 * aggregator are serialised by an internal mutex.  If a launch that
 * hydro_submit triggers fails (HYDRO_EHIP), the task stays held with its
 * ticket set and a later flush retries it.  A ticket identifies one
 * task; its result (amax of the sub-grid) is retrieved once, by hydro_poll
 * (non-blocking) or hydro_wait (blocking).  hydro_agg_destroy launches held
 * tasks and waits for all work.
 */
typedef struct hydro_agg hydro_agg_t;

typedef struct {
  uint64_t submitted, batches, launched;
  uint64_t flush_width, flush_idle, flush_timeout, flush_manual;
  uint64_t refused;            /* HYDRO_EAGAIN answers                        */
  uint64_t width_hist[11];     /* batches of width 1, 2-3, 4-7, ..., >= 1024  */
  uint64_t held, held_bytes;   /* tasks held now; output bytes held+in flight */
} hydro_agg_stats_t;

int hydro_agg_create(hydro_agg_t **out, int32_t max_width, double timeout_us,
                     int32_t n_streams, uint64_t hbm_budget_bytes,
                     int32_t flush_when_idle);
int hydro_submit(hydro_agg_t *agg, const hydro_subgrid_t *sg, double dt,
                 double dx, uint64_t *ticket);
/* hydro_submit_many: count tasks submitted in order, exactly as count
 * hydro_submit calls would be (each may trigger a launch by the rules above;
 * this is how a burst of tasks reaches the aggregator without a host call
 * per task).  tickets: count uint64_t, or NULL for fire-and-forget tasks
 * whose completion records are dropped when their batch completes (their
 * tickets are unknown to poll/wait; use hydro_agg_drain).  *submitted
 * receives the number of tasks taken; HYDRO_EAGAIN when admission stops the
 * burst (the rest were not submitted).  Errors as hydro_submit. */
int hydro_submit_many(hydro_agg_t *agg, const hydro_subgrid_t *sg,
                      int32_t count, double dt, double dx, uint64_t *tickets,
                      int32_t *submitted);
/* hydro_agg_drain: launch whatever is held and wait for every batch in
 * flight (results of tasks with tickets stay retrievable). */
int hydro_agg_drain(hydro_agg_t *agg);
int hydro_flush(hydro_agg_t *agg);     /* launch whatever is held now        */
int hydro_progress(hydro_agg_t *agg);  /* collect completions; apply the
                                          timeout / idle-stream rules        */
int hydro_poll(hydro_agg_t *agg, uint64_t ticket, int32_t *done, double *amax);
int hydro_wait(hydro_agg_t *agg, uint64_t ticket, double *amax);
int hydro_agg_stats(hydro_agg_t *agg, hydro_agg_stats_t *out);
int hydro_agg_destroy(hydro_agg_t *agg);

/*
 * Serving loop (continuous batching on device-resident state).  `pool` holds
 * resident sub-grids (u_in used; u_out ignored).  Task i steps sub-grid
 * task_subgrid[i] and arrives at arrival_us[i] (microseconds after the loop
 * starts, non-decreasing; the caller draws them, e.g. Poisson).  An arrived
 * task is admitted as soon as an output slab of its edge class is free
 * (slabs[e] slabs at slab_base[e] for n = 8, 12, 16 -- the HBM budget of the
 * loop; a slab is nfields x (n+6)^3 doubles with out_layout STORED, nfields x
 * n^3 with INTERIOR, so the same budget holds more tasks), is submitted to an
 * aggregator configured by cfg, and releases its slab when its batch has
 * completed (unless keep_slabs).  Per task the loop reports latency_us =
 * completion observed - arrival, and optionally amax and the slab used.
 * Runs on the calling thread until every task has completed.
 */
typedef struct {
  int32_t max_width;
  double timeout_us;
  int32_t n_streams;
  int32_t flush_when_idle;
  int32_t nfields;
  double dt, dx;
  double *slab_base[3];
  int32_t slabs[3];
  int32_t keep_slabs;
  int32_t out_layout;   /* layout of the output slabs: HYDRO_OUT_STORED/INTERIOR */
} hydro_serve_config_t;

typedef struct {
  hydro_agg_stats_t agg;
  double makespan_us;      /* last completion, from loop start             */
  double first_admit_us;
  uint64_t max_live;       /* most tasks admitted and not yet completed    */
  uint64_t slab_waits;     /* loop passes where an arrived task had no slab */
  double launch_host_us;   /* host time in batch launches (runtime calls)  */
} hydro_serve_stats_t;

int hydro_serve_run(const hydro_serve_config_t *cfg, const hydro_subgrid_t *pool,
                    int32_t pool_count, const int32_t *task_subgrid,
                    const double *arrival_us, int32_t ntasks, double *latency_us,
                    double *amax_out, double **out_slab, hydro_serve_stats_t *stats);

/*
 * Width cost model: a 5-64-64-1 FP32 perceptron with ReLU that predicts the
 * (standardised, log) p99 latency of a serving condition at an aggregation
 * width, trained on the GPU by these kernels; the width with the lowest
 * prediction is chosen (it replaces hand-sweeping the paper's "max aggregated
 * kernels" parameter, Section VI-B).  All pointers are device pointers.
 * params: HYDRO_MLP_PARAMS floats laid out W1[64][5] b1[64] W2[64][64] b2[64]
 * W3[64] b3.  x: rows x 5 features, row-major.  act: 2 x rows x 64 floats
 * (hidden activations, written by the forward pass when not NULL and needed
 * by the backward pass).  scratch: 2 x rows x 64 floats.  grad: HYDRO_MLP_
 * PARAMS floats (overwritten, not accumulated).  Reductions run in a fixed
 * order: results are deterministic.  Nothing is allocated.
 */
#define HYDRO_MLP_INPUTS 5
#define HYDRO_MLP_HIDDEN 64
#define HYDRO_MLP_PARAMS 4609
int hydro_mlp_forward(const float *params, const float *x, int32_t rows, float *y,
                      float *act, void *stream);
int hydro_mlp_backward(const float *params, const float *x, const float *act,
                       const float *dy, int32_t rows, float *scratch, float *grad,
                       void *stream);
/* loss = mean((y - target)^2) (device scalar, may be NULL); dy = 2 (y - target)/rows */
int hydro_mlp_mse(const float *y, const float *target, int32_t rows, float *dy,
                  float *loss, void *stream);
/* one Adam step (bias-corrected, step >= 1) over n parameters */
int hydro_mlp_adam(float *params, const float *grad, float *m, float *v, int32_t n,
                   float lr, float beta1, float beta2, float eps, int32_t step,
                   void *stream);

/*
 * hydro_math_check -- diagnostic: evaluates, on the device, the reciprocal
 * and reciprocal-square-root routines every hydro kernel uses (1/rho in the
 * primitive recovery, the sound speed sqrt(gamma p / rho) =
 * gamma p / sqrt(gamma p rho) and the 1/(a+ - a-) of the central-upwind
 * flux, Section IV-B) on n caller-given arguments, so that tests can bound
 * their error against correctly rounded results.
 *   x          device, n doubles, each positive and normal.
 *   recip_out  device, n doubles: recip(x[i]) ~ 1/x[i].
 *   rsqrt_out  device, n doubles: rsq(x[i]) ~ 1/sqrt(x[i]).
 * Errors: HYDRO_EINVAL for n < 0 or a NULL pointer with n > 0; HYDRO_EHIP if
 * the launch fails.  Enqueues on `stream` (NULL = default stream).
 */
int hydro_math_check(const double *x, int32_t n, double *recip_out, double *rsqrt_out,
                     void *stream);

/* Thread-local text of the last error on the calling thread ("" if none). */
const char *hydro_last_error(void);

/* Library build string: target, a hash of every library source ("src X")
 * and a hash of the hydro kernels' sources and compile flags ("kernels Y"),
 * which changes only when their machine code can.  Static storage. */
const char *hydro_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HYDROAGG_H */
