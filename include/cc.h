/*
 * cc.h -- C ABI of the MI355X cut-cell library (libcutcell.so).
 *
 * One dimensionally split finite-volume step of the 2D Euler equations on a uniform
 * Cartesian grid around a rigid convex body that moves every step, with the moving-
 * boundary flux stabilisation of Bennett, Nikiforakis & Klein (arXiv:1711.11361):
 *   - cut-cell geometry of the body at the old, intermediate and new time levels
 *     (Sec. 2.1: volume fractions; Sec. 2.2: face apertures and shielded volumes;
 *      Sec. 2.3.4: time-averaged apertures, Eq. timeAveragedBeta);
 *   - per sweep: MUSCL-Hancock + HLLC "standard" fluxes on every face, a moving-wall
 *     Riemann problem per cut cell (Eq. riemann_wallvel), the stabilised shielded fluxes
 *     (Eqs. Klein2shieldedFluxMethod2, ModifiedBoundaryFluxMethod2,
 *      Klein2DtotalfluxaMethod2), the conservative update
 *     (Eqs. Klein2DcompleteMovingMethod2a/b) and the treatment of cells that are
 *     uncovered or covered (Eqs. volumeWeighting ... cutCellCoverDonation, Sec. 2.3.5);
 *   - sweeps alternate x-y / y-x from step to step (Sec. 2.3.4, end);
 *   - a global CFL time step from the regular cell size (Sec. 4).
 *
 * Conventions
 *   Memory: the caller allocates every device byte.  cc_workspace_bytes() gives the exact
 *     size of the workspace passed to cc_create(); the library never allocates device
 *     memory.  Host pointers are read only during the call.
 *   Layout: fields are structure-of-arrays planes of nx*ny values, row-major (index
 *     j*nx + i, cell (i, j) spans [x_lo + i hx, x_lo + (i+1) hx] x [...]).  Conserved
 *     planes are (rho, rho u, rho v, E) per unit CELL volume (U = alpha Q); primitive
 *     planes are (rho, u, v, p).
 *   Streams: every call is asynchronous on the stream given to cc_create() unless it
 *     returns host data (cc_cfl_dt, cc_totals, cc_info, cc_timing_read), which
 *     synchronises that stream.
 *   Errors: functions return cc_status and never abort.  Argument errors are detected
 *     synchronously; device-detected state errors (no donor for a cell that becomes
 *     fluid, non-finite or non-physical states) are reported by the next synchronising
 *     call.  cc_last_error() gives a message.
 *   Threads: one context must not be used from two host threads at once.
 */
#ifndef CC_H
#define CC_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cc_ctx cc_ctx; /* opaque */

typedef enum {
    CC_OK = 0,
    CC_ERR_ARG = 1,         /* invalid argument or call order */
    CC_ERR_DEVICE = 2,      /* HIP runtime error */
    CC_ERR_WORKSPACE = 3,   /* workspace too small, or the body outgrew the staging capacity */
    CC_ERR_STATE = 4,       /* non-finite/non-physical state, or a cut cell left inadmissible */
    CC_ERR_MOTION = 5,      /* the body moves one cell or more within a sweep, or dt <= 0 */
    CC_ERR_UNSUPPORTED = 6
} cc_status;

typedef enum { CC_FP64 = 0, CC_FP32_GEOM64 = 1 } cc_precision;
typedef enum { CC_BC_TRANSMISSIVE = 0, CC_BC_REFLECTIVE = 1 } cc_bc;

typedef struct {
    int32_t nx, ny;
    int32_t bc[4];      /* W, E, S, N (cc_bc) */
    int32_t precision;  /* cc_precision: FP64 state, or FP32 state and dense fluxes with FP64
                           geometry and FP64 cut-cell arithmetic */
    int32_t options;    /* bit 0: axisymmetric about the x axis (y is the radius, y_lo >= 0; the
                           geometric source of the axisymmetric Euler equations, Sec. 3.5, is applied
                           before each step's first sweep; reading R33); other bits must be 0 */
    double x_lo, x_hi, y_lo, y_hi;
    double gamma;       /* ratio of specific heats (perfect gas, Sec. 2.1) */
    double alpha_min;   /* small-cell threshold: a cut cell whose volume fraction is below it
                           counts as solid (alpha = 0), so it is covered and uncovered like any
                           solid cell (Eqs. cutCellCoverDonation, cutCellInitialisation); 0 keeps
                           every cut cell (the paper's method, whose update divides by the new
                           volume fraction, Eq. EulerDiscrete2); must lie in [0, 0.5) */
} cc_config;

typedef struct {
    int32_t nverts;      /* 0: no body */
    int32_t pad_;
    const double* verts; /* body-frame convex polygon, counter-clockwise, (x, y) pairs, at most
                            2048 vertices (CC_ERR_UNSUPPORTED beyond); host */
    double ref_x, ref_y; /* position of the body-frame origin at t = 0 */
    double theta0;       /* body angle at t = 0 (radians, counter-clockwise) */
    double vx, vy;       /* constant translation velocity */
    double pitch_amp, pitch_omega; /* theta(t) = theta0 + pitch_amp sin(pitch_omega t) */
} cc_body;

/* Exact device bytes needed by cc_create() for this grid and body (state, three geometry
 * levels, staging for the body's region, reductions). */
size_t cc_workspace_bytes(const cc_config* cfg, const cc_body* body);

/* Create a context on the current device.  d_ws: device workspace of ws_bytes (>=
 * cc_workspace_bytes), 256-byte aligned, owned by the caller until cc_destroy().
 * hip_stream: a hipStream_t (NULL = default stream). */
cc_status cc_create(const cc_config* cfg, const cc_body* body, void* d_ws, size_t ws_bytes, void* hip_stream,
                    cc_ctx** out);
cc_status cc_destroy(cc_ctx* ctx);

/* Several bodies in one context: the sloped channel of Sec. 3.1 (its two walls are two
 * solid regions moving together) and bodies in relative motion (Sec. 3.5, planar).  The
 * solid region is the union of the bodies' closed polygons (each as for cc_body: convex,
 * counter-clockwise, here with 3 to 256 vertices), each posed with its own motion.
 * Reading R30 (the paper describes the method for one convex body): vertex solid when in
 * any body; a face's solid interval from the one body that meets it; volume fraction one
 * minus the sum of the bodies' areas in the cell; a wall cell takes the velocity of the
 * body that cuts it; the exact time-averaged aperture of a face sums the bodies' swept
 * areas, each over its own displacement.  The bodies must keep apart: a face or cell with
 * solid parts of two bodies, or a wall cell cut by different bodies at a sweep's two
 * levels, sets device status bit 4, and the next synchronising call returns
 * CC_ERR_UNSUPPORTED.  nbodies 0 or 1 is cc_create (bodies: NULL, or one body).  With
 * two or more, the geometry and box phases cover the whole grid, and steps are planned on
 * the host: cc_advance, the persistent launch mode, batches, cc_autotune and
 * cc_surface_loads (use cc_body_loads) return CC_ERR_UNSUPPORTED.  bodies: host,
 * copied; at most CC_MAX_BODIES. */
#define CC_MAX_BODIES 4
size_t cc_workspace_bytes_bodies(const cc_config* cfg, const cc_body* bodies, int32_t nbodies);
cc_status cc_create_bodies(const cc_config* cfg, const cc_body* bodies, int32_t nbodies, void* d_ws, size_t ws_bytes,
                           void* hip_stream, cc_ctx** out);

/* Initial state: body posed at time t0, level-n geometry built, U = alpha Q(prim); the
 * clock starts at t0, step 0.  Also valid on a context that has already been stepped:
 * every geometry slot is rebuilt at t0, so the run starts as on a fresh context.
 * d_prim: device, 4 planes (rho, u, v, p) of nx*ny doubles. */
cc_status cc_set_state(cc_ctx* ctx, const double* d_prim, double t0);
/* Resume the clock (restart from a saved state): time t after `step` completed split steps.
 * The next step sweeps x then y if `step` is even, y then x if odd (the alternation of
 * Sec. 2.3.1), and the geometry (level n and the other two slots) is rebuilt with the body
 * posed at t, so a state saved from an uninterrupted run continues bit for bit.  The state itself is unchanged:
 * set it afterwards with cc_set_u.  Errors: CC_ERR_ARG for step < 0 or non-finite t. */
cc_status cc_set_clock(cc_ctx* ctx, double t, int64_t step);
/* Replace the conserved state (device, 4 planes of nx*ny doubles, per unit cell volume). */
cc_status cc_set_u(cc_ctx* ctx, const double* d_u);
/* Copy the level-n state out: what = 0 primitive (rho, u, v, p; zeros in solid or empty
 * cells), what = 1 conserved U.  d_out: device, 4*nx*ny doubles. */
cc_status cc_get_state(cc_ctx* ctx, double* d_out, int32_t what);

/* Cut-cell geometry of the body posed at time t into a level: level 0 = level n (the one
 * the state refers to), 1 = stage level, 2 = level n+1. */
cc_status cc_geometry(cc_ctx* ctx, double t, int32_t level);
/* Copy a level out (device pointers, any may be NULL): vertex classes (int8,
 * (ny+1)*(nx+1), 1 = solid), volume fractions (nx*ny), x-face apertures (ny*(nx+1)),
 * y-face apertures ((ny+1)*nx), and the cut-cell list (Sec. 2.1: cells the wall cuts, here
 * the cells whose four faces are neither all open nor all closed): d_cut (int32, room for
 * nx*ny entries) receives their linear indices j*nx + i in increasing order and d_ncut (one
 * int32) their number; give both or neither (CC_ERR_ARG).  Asynchronous. */
cc_status cc_geometry_dump(cc_ctx* ctx, int32_t level, int8_t* d_vcls, double* d_alpha, double* d_bx,
                           double* d_by, int32_t* d_cut, int32_t* d_ncut);

/* Split step in parts: cc_begin_step poses the body at t + dt and builds the stage level
 * (the first sweep's direction moves the polygon, the other coordinate stays) and level
 * n+1; cc_sweep runs the next sweep (dir 0 = x, 1 = y; x first on even steps, y first on
 * odd steps); cc_end_step makes level n+1 the new level n and advances time. */
cc_status cc_begin_step(cc_ctx* ctx, double dt);
cc_status cc_sweep(cc_ctx* ctx, int32_t dir, double dt);
cc_status cc_end_step(cc_ctx* ctx);
/* One full split step of size dt. */
cc_status cc_step(cc_ctx* ctx, double dt);

/* Global time step (Sec. 4: from the regular cell size) dt = cfl * min(hx / Sx, hy / Sy),
 * S the largest signal speed |u|+a over live cells and |u_wall| over the body's vertices.
 * h_dt (host, nullable): written after synchronising; errors of the state are returned.
 * d_dt (device, nullable): written asynchronously on the context's stream, the same value
 * bit for bit, or 0 when the state is not finite or the status word reports an error (the
 * error surfaces at the next synchronising call).  At least one of them (CC_ERR_ARG). */
cc_status cc_cfl_dt(cc_ctx* ctx, double cfl, double* h_dt, double* d_dt);

/* nsteps CFL steps planned on the device (Sec. 4 time step, Sec. 2.3.4 poses): each step
 * takes dt = cfl * min(hx / Sx, hy / Sy) from the state it starts from, exactly as
 * cc_cfl_dt, then runs the split step as cc_step; a block at the head of every step
 * computes dt, the poses, regions and sweep boxes on the device, so the host queues all
 * steps without waiting between them.  Results equal those of cc_cfl_dt + cc_step bit for
 * bit for a body that does not turn (a turning body's angle uses the device's sin and
 * cos).  Host outputs, each nullable: h_dt (nsteps doubles) the steps' dt, h_step_ms
 * (nsteps floats) each step's device time from events between the steps, h_done the steps
 * completed.  Stops at the first step that cc_cfl_dt or cc_step would refuse, with the
 * same status (the state is then that after the last completed step).  Uses the per-phase
 * launches whatever the launch mode.  Not for a context in a batch.  Synchronizes. */
cc_status cc_advance(cc_ctx* ctx, int32_t nsteps, double cfl, double* h_dt, float* h_step_ms, int32_t* h_done);

/* Surface loads at level n (post-processing of the pitching aerofoil of Sec. 3.6): the sum
 * over cells with fluid content of p* N, where p* is the wall pressure of the wall Riemann
 * problem (Eq. riemann_wallvel, HLLC with Davis speeds, reading R9) between the cell state
 * U/alpha and its mirror image moving with the body at the cell's wall point, and N the
 * level's effective wall normal ((beta_W - beta_E) hy, (beta_S - beta_N) hx), pointing
 * into the body (reading R12).  h_out4 (host, 4 doubles): Fx, Fy, the moment Mz about the
 * body's pose origin, and sum p* |N| (the scale against which the rounding of the other
 * three is measured).  Deterministic summation order; zeros without a body.  Needs a state
 * and no open step (CC_ERR_ARG).  Synchronizes.  A context with several bodies: CC_ERR_UNSUPPORTED
 * (see cc_body_loads). */
cc_status cc_surface_loads(cc_ctx* ctx, double* h_out4);

/* The same loads on one body of a context with several bodies (cc_create_bodies; reading R30):
 * the sum over the wall cells that body cuts at level n, each with its own wall velocity, and
 * the moment about that body's pose origin.  body: 0 .. nbodies - 1 (a one-body context takes
 * 0 and returns cc_surface_loads); CC_ERR_ARG otherwise.  Synchronizes. */
cc_status cc_body_loads(cc_ctx* ctx, int32_t body, double* h_out4);

/* Wall pressure distribution at level n (the surface pressure of the pitching aerofoil,
 * Sec. 3.6; from it the pressure coefficient of each wall cell): for every cell with fluid
 * content and a non-zero effective wall normal, in increasing linear index j nx + i, six
 * doubles: that index, the wall point x and y, p* of the wall Riemann problem (Eq.
 * riemann_wallvel, reading R9) and the normal N (Nx, Ny; |N| the wall length, pointing into
 * the body) -- the terms whose sums cc_surface_loads returns.  d_out (device, caller-owned,
 * 6 * max_records doubles; may be null when max_records is 0) receives the first
 * max_records records; *h_n (host) the number of wall cells, also when it exceeds
 * max_records (call with 0 to size the buffer).  With several bodies, every body's wall cells,
 * each p* with the velocity of the body that cuts the cell.  Synchronizes. */
cc_status cc_surface_pressure(cc_ctx* ctx, double* d_out, int32_t max_records, int32_t* h_n);

/* Conservation totals sum(U) hx hy per component (rho, rho u, rho v, E), FP64,
 * deterministic order, into h_totals4 (host).  h_budget12 (host, nullable): the
 * conservation budget since cc_set_state (Sec. 3.3, mass-conservation error), zeros unless
 * cc_set_budget switched it on: [0..3] the fluxes through the domain boundary (dt/h times
 * the stabilised face fluxes of the first and last face of every line, in minus out, times
 * the cell area), [4..7] the wall terms of the cut cells (dt/h times
 * (beta_hi - beta_lo)(F^B - u_wall Q^B) times the cell area), [8..11] the
 * residuals of emptied cells that found no recipient (times the cell area).  The totals
 * then change by boundary + wall - lost: with FP64 state to round-off, with FP32 state up to
 * the state's rounding (the mass drift).  Synchronises. */
cc_status cc_totals(cc_ctx* ctx, double* h_totals4, double* h_budget12);

/* Track the conservation budget (on = 1) or not (0, the default).  Switching it on resets
 * the running sums.  Tracking costs a few writes per boundary cell and a longer collapse
 * launch per sweep; it is not available in the persistent launch mode
 * (CC_ERR_UNSUPPORTED).  Synchronises. */
cc_status cc_set_budget(cc_ctx* ctx, int32_t on);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the totals of cc_totals for a state
 * held outside any context, computed by the same kernels in the same order (so the two
 * agree bit for bit for the same state), written to device memory.  It allocates nothing:
 * the partial sums go to a scratch array of 4 x 1024 doubles (32 KiB) that the library
 * keeps in each device's memory from the first call on that device until the process
 * ends.  All calls on one device share that array, so calls that overlap in time on one
 * device (from different streams or threads) race: serialise them.
 *   d_u: device, 4 planes (rho, rho u, rho v, E per unit cell volume) of nx*ny values,
 *        FP64 for precision CC_FP64, FP32 for CC_FP32_GEOM64; read only;
 *   hx, hy: cell sizes (the totals are sums times hx hy);
 *   hip_stream: a hipStream_t of the current device (NULL = default stream);
 *   d_out4: device, 4 doubles, written asynchronously on hip_stream.
 * Returns at once (asynchronous).  CC_ERR_ARG for null pointers, sizes below 1 or an
 * unknown precision; CC_ERR_UNSUPPORTED above CC_TOTALS_STATE_MAX_CELLS cells;
 * CC_ERR_DEVICE if the launch fails.  cc_last_error(NULL) gives the message. */
#define CC_TOTALS_STATE_MAX_CELLS 2147483647
cc_status cc_totals_state(const void* d_u, int32_t precision, int32_t nx, int32_t ny, double hx, double hy,
                          void* hip_stream, double* d_out4);

/* Host info vector (n entries used, up to 11): time, steps, parity, device status bits
 * (1: a cell turned fluid, or was emptied, with no donor next to it — reported only: the
 * cell keeps no content until a donor appears; 2: a cell stayed inadmissible after
 * collapsing; 4: two of several bodies met in one face or cell; 8: a grid-barrier wait of
 * a persistent launch ran out; 2, 4 and 8 are errors),
 * collapsed-cell count, sweep box cells of the last sweep, staging capacity, rows per block
 * of the dense x-sweep, rows per tile of the dense y-sweep, 1 if that sweep walks columns
 * (else 0), 1 if an x sweep's dense launch also runs the box cells' first phase (small
 * grids; else that phase has a launch of its own before it; a y sweep's dense launch always
 * runs it).  Synchronizes. */
cc_status cc_info(cc_ctx* ctx, double* h_out, int32_t n);

/* Tile tuner for the dense sweeps (the regular cells): times every tile shape of both
 * sweeps on this grid, reps launches each (as a step launches them: beside the first box
 * phase), from the current state into the spare state buffer, and keeps the fastest for
 * this context (the current variant unless another is at least 3 % faster).  h_choice
 * (nullable, host, 2 entries) receives the chosen variant indices.  cache_path (nullable):
 * a text file of earlier choices, one line "key tile_x tile_y" per configuration (the key
 * names the device, the precision and the grid); a configuration found there is applied
 * without timing, a new choice is appended.  Needs a state and no open step (CC_ERR_ARG).
 * Synchronizes; results do not depend on the choice (every shape computes the same
 * values, bit for bit). */
cc_status cc_autotune(cc_ctx* ctx, int32_t reps, int32_t* h_choice, const char* cache_path);
/* Set the dense-sweep tile variants directly: tile_x indexes rows per x-sweep block
 * {1, 2, 4, 8}; tile_y 0-3 rows per 64-column y-sweep tile staged in LDS {8, 12, 16, 24}
 * (16 and 24 only with FP32 state: the tile lives in 64 KiB of LDS), 4-5 column walks of
 * 256 columns x {4, 8} rows with the states in registers (8 only with FP32 state).  CC_ERR_ARG for an index out
 * of range. */
cc_status cc_set_tiles(cc_ctx* ctx, int32_t tile_x, int32_t tile_y);

/* How cc_step launches a whole step (results are identical, bit for bit, in both modes).
 * CC_LAUNCH_PER_PHASE (default): every phase is one kernel launch, the step one captured
 * HIP graph.  CC_LAUNCH_PERSISTENT: one launch per sweep whose phases are separated by
 * grid-wide barriers, the dense tiles overlapping the cut-cell phases (tile variants 0-1
 * only; other variants fall back to the per-phase launches).  Each barrier wait is bounded
 * in time; a wait that runs out sets status bit 8 and the step reports CC_ERR_DEVICE.
 * CC_ERR_ARG for an unknown mode or inside a step.  Synchronizes. */
typedef enum { CC_LAUNCH_PER_PHASE = 0, CC_LAUNCH_PERSISTENT = 1 } cc_launch_mode;
cc_status cc_set_launch_mode(cc_ctx* ctx, int32_t mode);

/* Timing with HIP events on the context's stream.  mode bit 0: cc_step issues the
 * captured step's launches one by one (same kernels, grids and arguments) and each dense
 * launch (the merged first box phase and dense tiles) records its own start/stop events
 * (no extra stream commands, so the interval is that kernel's execution); single sweeps
 * (cc_sweep) time their separate dense launches the same way.  Bit 1: cc_step runs single
 * sweeps and events bracket their box-kernel and geometry phases (extra stream commands).
 * 0 stops recording.  cc_timing_read returns, since the last read, pairs (total ms,
 * count) for: dense x, dense y, box phases, geometry (8 doubles). */
cc_status cc_timing(cc_ctx* ctx, int32_t mode);
cc_status cc_timing_read(cc_ctx* ctx, double* h_out, int32_t n);

const char* cc_last_error(const cc_ctx* ctx);

/* ------------------------------------------------------------------------- batches
 * A batch steps many contexts of one precision together: every phase of the split step
 * is one kernel launch over all members (grids sized from each member's capacities, so a
 * whole step is one captured HIP graph, replayed while the membership is unchanged).
 * Members keep their own workspaces, state, clock and step order; a context in a batch
 * is stepped only through it (cc_step, cc_begin_step and cc_autotune refuse).
 * Membership may change between steps (continuous batching). */
typedef struct cc_batch cc_batch; /* opaque */

/* Device bytes for a batch of up to max_instances members (argument blocks, launch
 * tables, read-back areas). */
size_t cc_batch_workspace_bytes(int32_t max_instances);
/* Create on the given stream (a hipStream_t, not the null stream, so that steps can be
 * captured).  d_ws: device, >= cc_batch_workspace_bytes, 256-byte aligned, owned by the
 * caller.  precision: cc_precision of every member.  CC_ERR_ARG / CC_ERR_WORKSPACE /
 * CC_ERR_DEVICE on failure. */
cc_status cc_batch_create(int32_t max_instances, int32_t precision, void* d_ws, size_t ws_bytes, void* hip_stream,
                          cc_batch** out);
cc_status cc_batch_destroy(cc_batch* b);
/* Add a context with a state set and no open step (synchronizes its stream); CC_ERR_ARG
 * if it is in a batch or of another precision, CC_ERR_WORKSPACE if the batch is full. */
cc_status cc_batch_add(cc_batch* b, cc_ctx* ctx);
cc_status cc_batch_remove(cc_batch* b, cc_ctx* ctx);
int32_t cc_batch_size(const cc_batch* b);
/* Dense-sweep tile variants used by every member (as cc_set_tiles). */
cc_status cc_batch_set_tiles(cc_batch* b, int32_t tile_x, int32_t tile_y);
/* Tile tuner for the batch's dense launches (as cc_autotune, with every member's grid in
 * the launches and in the cache key, in membership order).  Needs members (CC_ERR_ARG).
 * Synchronizes. */
cc_status cc_batch_autotune(cc_batch* b, int32_t reps, int32_t* h_choice, const char* cache_path);
/* Launch mode of the batch's steps (as cc_set_launch_mode). */
cc_status cc_batch_set_launch_mode(cc_batch* b, int32_t mode);
/* One split step of every member, member k with time step h_dt[k] (host, in membership
 * order).  Also reduces each member's wave speeds for its next step and gathers the
 * status words; synchronizes.  h_status (nullable, host): each member's status bits. */
cc_status cc_batch_step(cc_batch* b, const double* h_dt, int32_t* h_status);
/* Next time steps from the wave speeds the last cc_batch_step reduced (no device work);
 * a member whose state is not finite or whose status is set gets 0 and its bits in
 * h_status (nullable). */
cc_status cc_batch_last_dt(cc_batch* b, double cfl, double* h_dt, int32_t* h_status);
/* Time steps from each member's current state (cc_cfl_dt per member). */
cc_status cc_batch_cfl_dt(cc_batch* b, double cfl, double* h_dt);
/* nsteps CFL steps of every member planned on the device, as cc_advance does for one
 * context (Sec. 4 time step, Sec. 2.3.4 poses), each member with its own time step, in one
 * launch per phase over all members; results equal those of the members advanced alone.
 * Host outputs, each nullable: h_dt (members x nsteps doubles, member-major) the time
 * steps, h_step_ms (nsteps floats) each step's device time, h_done (one per member) the
 * steps completed.  A member whose step would be refused stops there (its later steps do
 * nothing) while the others run on; the first such member's status is returned and
 * cc_batch_last_error names it.  Synchronizes. */
cc_status cc_batch_advance(cc_batch* b, int32_t nsteps, double cfl, double* h_dt, float* h_step_ms,
                           int32_t* h_done);
const char* cc_batch_last_error(const cc_batch* b);
/* Timing of a batch's steps (mode bit 0, as cc_timing: cc_batch_step issues the captured
 * step's launches one by one with events around each dense launch; 0 stops), and the
 * pairs (total ms, count) of dense x, dense y, box, geometry since the last read. */
cc_status cc_batch_timing(cc_batch* b, int32_t mode);
cc_status cc_batch_timing_read(cc_batch* b, double* h_out, int32_t n);

#ifdef __cplusplus
}
#endif
#endif /* CC_H */
