/*
 * nhswe.h -- C ABI of the MI355X (gfx950) time stepper for the
 * depth-integrated non-hydrostatic shallow-water system solved by the
 * projection-correction scheme of Escalante, Morales de Luna & Castro
 * (arXiv 1706.04551).
 *
 * One call of nh_step advances the state by one second-order TVD Runge-Kutta
 * step (Section 4.3 / Section 6: the projection-correction stage run twice and
 * averaged).  Each stage runs, on the device:
 *   - the second-order well-balanced PVM path-conservative finite-volume
 *     update of (h, hu, hv) with MUSCL-minmod reconstruction, desingularised
 *     velocities and the wet-dry treatment (Sections 4.1, 4.5, 5, eq. 16-22,30);
 *   - optionally the Manning friction of Section 2, semi-implicit, and the
 *     breaking terms of the eddy viscosity (Section 3, eq. 9-12);
 *   - walls, or outflow sides, and optional generation/absorption zones
 *     (Section 4.4);
 *   - the compact finite-difference non-hydrostatic pressure system at the
 *     cell corners: assembly (eq. 28-29, 37-41, 43), solve (Thomas in 1D,
 *     scheduled-relaxation Jacobi in 2D, eq. 32) and the correction of the
 *     discharges and of the vertical velocity w (eq. 26-28, 36, 41);
 * and the next time step comes from the CFL condition (eq. 23), reduced on the
 * device.
 *
 * Grid and layout.  nx x ny cells of size dx x dy; ny == 1 selects the 1D
 * channel of Section 4.  Host arrays passed through this interface are FP64,
 * row-major, x fastest:
 *   cells   [ny][nx]                  h, hu, hv, H (still-water depth, > 0 in
 *                                     water, <= 0 on dry land)
 *   corners [ny+1][nx+1] (1D: [nx+1]) w (depth-averaged vertical velocity),
 *                                     p (non-hydrostatic bottom pressure)
 * Corner (k, l) sits at x = k dx, y = l dy.  Walls bound the domain on every
 * side unless a side is open or a direction periodic (nh_params).
 *
 * Ownership.  The solver owns its device buffers, except those it borrows
 * through nh_bind_device_buffers.  Host arrays are always owned by the caller
 * and are copied in (set_*) or out (read_state); the state stays in device
 * memory between steps.
 *
 * Errors.  Every call returns an nh_status; no exception crosses the ABI.
 * nh_last_error() returns a thread-local message for the last failing call.
 * A step that fails (non-finite state) leaves the solver in NH_ESTATE until
 * the next nh_set_state.
 *
 * Threading.  A solver is bound to one HIP stream and is not thread-safe;
 * different solvers may be used from different threads.
 */
#ifndef NHSWE_H
#define NHSWE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NH_OK = 0,
  NH_EINVAL = -1,      /* bad argument (sizes, parameters, null pointer) */
  NH_ENOMEM = -2,      /* device allocation failed */
  NH_EDEVICE = -3,     /* HIP runtime error */
  NH_ENOCONV = -4,     /* pressure solve reached solve_max_iter */
  NH_ENONFINITE = -5,  /* NaN or Inf in the state after a step */
  NH_ENEGDEPTH = -6,   /* negative depth passed to nh_set_state */
  NH_ESTATE = -8       /* solver not ready (no state / failed earlier) */
} nh_status;

enum { NH_FP64 = 0, NH_FP32 = 1 };

typedef struct nh_solver nh_solver;

typedef struct {
  int32_t nx, ny; /* cells; ny == 1: 1D channel */
  double dx, dy;  /* cell sizes [m] (dy ignored in 1D) */
} nh_grid;

typedef struct {
  double g;            /* gravity [m/s^2] */
  double cfl;          /* CFL number of eq. (23), 0 < cfl <= 1 */
  double delta;        /* desingularisation depth of Section 4.5 (1e-5) */
  double dry_eps;      /* h <= dry_eps is dry (1e-10 FP64, 1e-5 FP32) */
  int32_t precision;   /* NH_FP64, or NH_FP32: bulk state and stencils in
                          FP32; solver residuals, convergence measure and
                          dt in FP64 */
  int32_t nh_on;       /* 0: hydrostatic shallow water only */
  int32_t breaking_on; /* eddy-viscosity breaking terms (Section 3) */
  double b1, b2;       /* breaking coefficients of eq. (9) */
  int32_t solve_max_iter; /* cap on relaxation sweeps per solve (2D) */
  int32_t check_every;    /* convergence measure every this many sweeps; a
                             multiple of n_omega */
  double solve_tol;    /* stop when max_c |(rhs - A p)_c / diag_c| < tol, the
                          size of a plain Jacobi update (eq. 32) */
  const double *omega_schedule; /* relaxation factors applied cyclically,
                                   copied at create; NULL => {1.0} */
  int32_t n_omega;
  int32_t fixed_dt;    /* 1: every step uses dt below instead of the CFL */
  double dt;
  double manning;      /* Gauckler-Manning n of the friction law of Section 2
                          [s m^-1/3], >= 0; 0: no friction.  Applied
                          semi-implicitly to each stage's finite-volume
                          result in wet cells: q <- q / (1 + dt g n^2 |u| /
                          h^(4/3)), |u| from the desingularised velocities.
                          Ensemble members may differ in it; the adjoint
                          covers it */
  int32_t open_sides;  /* outflow boundaries (Section 4.4), a bit per side:
                          1 west (x = 0), 2 east, 4 south (y = 0), 8 north
                          (south/north ignored in 1D).  An open side has
                          homogeneous Neumann ghosts that copy the adjacent
                          cell (h, H and both discharges); p is even across
                          it, as at a wall.  Unset sides are walls.  The
                          adjoint needs 0 */
  int32_t periodic;    /* periodic directions (Section 4.4, item 1), a bit
                          each: 1 x, 2 y (ignored in 1D).  The first and last
                          cells of a periodic line are neighbours: ghosts
                          wrap around, discharges keep their sign, the
                          pressure rows reach across the seam (in 1D a cyclic
                          tridiagonal system, solved by the Sherman-Morrison
                          form of the Thomas algorithm).  The last corner of
                          a periodic line is its first: corner arrays keep
                          their [ny+1][nx+1] layout, both copies hold the
                          same values (give w and p that way).  A periodic
                          direction has no open side and no relaxation
                          zone; the adjoint needs 0 */
  int32_t w_advection; /* 0: the vertical velocity equation of the model,
                          h w_t = p (eq. 7); 1: the energy-consistent form
                          named after eq. 7, (hw)_t + div(hw u) = p, i.e.
                          h (w_t + u . grad w) = p: each stage's hyperbolic
                          step also carries w with the flow (first-order
                          upwind at the corners, corner velocity from the
                          means of q and h around the corner), before the
                          pressure step.  Single grids only (ensembles and
                          the adjoint need 0) */
  int32_t solve_path;  /* how a 2D pressure solve is launched (the results
                          are the same): 0 automatic -- one launch per solve
                          when the grid's tiles fit the co-resident
                          workgroups of the device (each keeps its tile's
                          rows on chip for the whole solve and decides on
                          convergence on the device; capped solves are then
                          reported at the next status read), else 1.  That
                          launch is a plain one of no more workgroups than
                          the device holds at once; should other work on the
                          device keep some of them waiting for longer than
                          the solve's bounded waits (seconds), the run
                          reports NH_EDEVICE;
                          1 launches of 8 sweeps, the convergence measure
                          read back by the host at each check;
                          2 the one launch per solve as a cooperative launch
                          (residency of every workgroup guaranteed by the
                          runtime, ~20 us more per solve), NH_EINVAL at
                          create when the grid does not fit.  Ensembles (all members
                          alike): 0 and 1 launches of 8 sweeps over every
                          member still active, the number of those read by
                          the host at each check; 2 one cooperative launch
                          per solve of all members (sweeps and checks as
                          phases between grid barriers, the host takes no
                          decision; at most 1024 members; NH_EINVAL at the
                          first run where cooperative launches are not
                          available).  The results are the same either way */
  int32_t solve_norm;  /* stop measure of a 2D relaxation solve: 0 the size
                          of a plain Jacobi update, max |(rhs - A p)/diag|
                          (eq. 32, solve_tol as stated above); 1 the
                          relative residual max |rhs - A p| / max |rhs| (the
                          absolute one when rhs = 0).  Single grids through
                          nh_create only (ensembles, the adjoint and
                          nh_run_noalloc need 0) */
  int32_t wait_polls;  /* polls of a wait between the workgroups of a
                          one-launch solve (single grid or ensemble) before
                          it gives up and the run reports NH_EDEVICE at its
                          next status read: 0 the default, 2^21 (seconds);
                          negative: every such wait gives up at once, which
                          exercises that path (tests).  An ensemble takes
                          its first member's */
} nh_params;

typedef struct {
  double t;             /* simulated time */
  double dt_next;       /* dt the next step will use */
  double dt_last;       /* dt of the last step */
  int64_t step;         /* steps taken since nh_set_state */
  int32_t sweeps[2];    /* relaxation sweeps of the two stages of the last
                           step */
  double measure;       /* convergence measure at the end of the last solve */
  int64_t sweeps_total; /* sweeps since nh_set_state */
  int64_t solves_total; /* pressure solves since nh_set_state */
  double clamped_mass;  /* mass added by the positivity clamp [m^3], summed
                           over the stages (the RK2 average keeps half of
                           it in the state) */
  int32_t last_status;
  double mass;          /* water volume sum h dx dy (1D: sum h dx) of the
                           state at the last status read [m^3] (0 right
                           after nh_set_state); a closed domain keeps
                           mass - clamped_mass / 2 constant */
  int64_t nondominant;  /* rows of the two pressure systems of the last step
                           that are not strictly diagonally dominant
                           (Gershgorin check of Section 5, |diag| against
                           the sum of the |off-diagonals|; reported, not
                           enforced: the paper checked dominance on its
                           cases, and steep free-surface curvature can lose
                           it).  FP32 bulk checks its FP32 rows */
  int64_t adjoint_sweeps; /* relaxation sweeps of the transposed solves of
                             the last nh_adjoint_run (both stages of every
                             step; 0 before one) */
} nh_stats;

/* Per-phase device time (ms) accumulated between events on the solver's
 * stream while profiling is on (nh_profile). */
typedef struct {
  double fv_ms;        /* finite-volume stages */
  double assemble_ms;  /* breaking + assembly of the pressure system */
  double solve_ms;     /* whole solves, including host convergence checks */
  double correct_ms;   /* corrections, RK average and dt reduction */
  int64_t fv_launches, assemble_launches, solve_launches, correct_launches;
  double sweep_kernel_ms;  /* back-to-back relaxation-sweep launches only */
  int64_t sweep_kernel_launches;
  int64_t sweep_kernel_sweeps; /* sweeps done by those launches */
  double sweep_kernel_corner_sweeps; /* corners x sweeps of those launches,
                                        summed over the grids they covered */
  double solve_kernel_ms;  /* one-launch solves only (solve_path): the
                              timed launches (every one with on = 1, both
                              solves of one step in n with on = n >= 2) */
  int64_t solve_kernel_launches;
  int64_t solve_kernel_sweeps; /* sweeps done by those launches */
} nh_profile_t;

/* Create a solver for the grid and parameters on `hip_stream` (a hipStream_t;
 * NULL = the solver creates its own).  Allocates all device memory. */
nh_status nh_create(const nh_grid *grid, const nh_params *params,
                    void *hip_stream, nh_solver **out);

/* Bathymetry H, cells [ny][nx] (host, FP64). */
nh_status nh_set_bathymetry(nh_solver *s, const double *H);

/* State: h, hu, hv cells (hv ignored in 1D, may be NULL = 0), w and p corners
 * (NULL = 0; p is the warm start of the first solve).  Resets t, step and
 * statistics and computes the first dt.  h must be >= 0 (NH_ENEGDEPTH). */
nh_status nh_set_state(nh_solver *s, const double *h, const double *hu,
                       const double *hv, const double *w, const double *p);

/* Generation/absorption zones (Section 4.4): after every step the state in a
 * zone is relaxed towards a target, U <- m U + (1 - m) U* in the cells, and
 * w and p likewise at the corners.  widths[4]: zone widths L [m] at the
 * west, east, south, north walls (0: no zone; south/north ignored in 1D).
 * Along one direction, the k + 1 cells nearest a wall with a zone (k the
 * least natural number with k dx >= L) get m = sqrt(max(0, 1 - (d/L)^2)),
 * d the distance to the zone's innermost cell, so m = 1 at its inner edge
 * and 0 at the wall cell; every other cell has m = 1.  In 2D the weights of
 * x and y multiply; a corner takes, per direction, the mean of the two
 * cells beside it (mirrored at a wall).  Targets, copied: h_t, q1_t, q2_t
 * over the cells (row-major ny x nx, h_t >= 0), w_t, p_t over the corners;
 * NULL gives still water (h* = max(H, 0), q* = w* = p* = 0: the absorbing
 * zone), so call nh_set_bathymetry first.  All widths 0 switches the zones
 * off.  NH_EINVAL for negative or non-finite widths or targets.  The
 * adjoint refuses a solver with zones. */
nh_status nh_set_relaxation(nh_solver *s, const double *widths,
                            const double *h_t, const double *q1_t,
                            const double *q2_t, const double *w_t,
                            const double *p_t);

/* Device memory owned by the caller (for instance PyTorch tensors) that the
 * solver borrows for the bathymetry and for the state U^n = (h, hu, hv) and
 * w of the scheme (Section 5, eq. 31), so that inputs and results need no
 * host copy.  Element type of the precision (double for NH_FP64, float for
 * NH_FP32), contiguous, row-major: H, h, hu, hv cells [ny][nx]; w corners
 * [ny+1][nx+1] ([nx+1] in 1D).  NULL = keep the current buffer.
 * Depth storage: an NH_FP64 grid stores the depth h in the h array; an
 * NH_FP32 (bulk) grid stores s = h - max(H, 0) there: over water (H > 0)
 * the surface elevation eta = h - H (its slopes and jumps, the well-balanced
 * pressure terms, are then differences of stored values instead of
 * differences of two nearly equal FP32 sums), on land (H <= 0) the depth
 * itself (thin films keep their digits); a dry cell holds -max(H, 0).  Host
 * arrays passed through nh_set_state / nh_read_state are always depths. */
typedef struct {
  void *H;
  void *h, *hu, *hv; /* hv: NULL in 1D */
  void *w;           /* NULL: w = 0 */
} nh_device_views;

/* Bind device views (see nh_device_views).  Each given view replaces the
 * solver's buffer for that array (a buffer the solver allocated is freed);
 * from then on the solver reads and writes it in place on its stream, so
 * after nh_step / nh_run it holds U^{n+1}, and nh_set_bathymetry,
 * nh_set_state and nh_read_state copy into and out of it.  Binding adopts
 * the contents: a bound H is the bathymetry (as nh_set_bathymetry); bound
 * h, hu (and hv in 2D), which go together, are the state as nh_set_state
 * would set it with that w (or w = 0, written into the current w buffer)
 * and p = 0: statistics reset and the first dt computed.
 * Ownership: the caller keeps the memory alive and leaves it untouched by
 * other streams while the solver's stream works on it, until nh_destroy or a
 * later bind of the same array.  Views are checked before anything changes:
 * NH_EINVAL for a view that is not device memory of the solver's device
 * (hipPointerGetAttributes), is misaligned, extends past its allocation,
 * overlaps another view, or holds non-finite values, and for an incomplete
 * state; NH_ENEGDEPTH for h < 0; NH_ESTATE for a state without bathymetry.
 * Synchronises the solver's stream. */
nh_status nh_bind_device_buffers(nh_solver *s, const nh_device_views *v);

/* One time step.  dt_used (nullable) receives the step's dt. */
nh_status nh_step(nh_solver *s, double *dt_used);

/* nsteps time steps, queued back to back; the device status (non-finite
 * state, no wet cell, and with one-launch solves a solve that reached
 * solve_max_iter) is read every 64 steps and at the end, and the run stops
 * there with the first failure found (NH_ENOCONV leaves the state valid). */
nh_status nh_run(nh_solver *s, int64_t nsteps);

/* Copy the state to the host (each pointer nullable). */
nh_status nh_read_state(nh_solver *s, double *h, double *hu, double *hv,
                        double *w, double *p);

nh_status nh_get_stats(const nh_solver *s, nh_stats *out);

/* Event timing on the solver's stream: 0 off; 1 every phase and every
 * back-to-back relaxation-sweep batch; n >= 2 only the sweep batch of one
 * cycle in n (phase fields stay 0), which leaves the step's time almost
 * untouched, whereas timing every phase adds ~13 % (each event pair stalls
 * the queue).  Turning it on clears the accumulated times. */
nh_status nh_profile(nh_solver *s, int32_t on);
nh_status nh_get_profile(nh_solver *s, nh_profile_t *out);

void nh_destroy(nh_solver *s);

/* ---- Adjoint -------------------------------------------------------------
 * Gradient of the gauge misfit
 *   J = 1/2 sum_{n=1..nsteps} sum_g (h^n_{gauge g} - target[n-1][g])^2
 * of a run of nsteps steps from the solver's current state, by the adjoint
 * (reverse) of the discrete time step: the transposed Jacobians of the
 * finite-volume update (eq. 20-22, 30), of the correction (eq. 36, 41) and of
 * the pressure system (eq. 37-41), whose solve is done with the transposed
 * five-point rows and the same relaxation schedule (eq. 32); every limiter,
 * speed and wet/dry decision is the forward run's.  The forward run is
 * checkpointed every ckpt_every steps and each segment is run again, with its
 * stage pressures recorded, before the adjoint goes back through it.
 *
 * Requires a 2D grid, a fixed time step (fixed_dt = 1), breaking_on = 0,
 * open_sides = 0 and no relaxation zones; Manning friction is covered.
 * gauges[ngauges]: flat cell indices j*nx + i; target[nsteps][ngauges] FP64.
 * adj_tol: a transposed solve stops when its measure of eq. (32) is below
 * adj_tol * max_c |pbar_c / diag_c| (pbar: its right-hand side).
 * Outputs (host, FP64, cells [ny][nx], each nullable except J): J; dJ/dh0,
 * dJ/dhu0, dJ/dhv0 w.r.t. the initial state at fixed bathymetry; dJ/dH w.r.t.
 * the bathymetry at fixed initial state.  For h0 = H + eta0 the gradient
 * w.r.t. eta0 is dJ/dh0 and that w.r.t. H at fixed eta0 is dJ/dH + dJ/dh0.
 * On return the solver holds the state after the nsteps forward steps.
 * Device memory: (nsteps/ckpt_every + 1) checkpoints and ckpt_every recorded
 * steps (3 cell and 1 corner arrays in the bulk type plus 2 FP64 corner
 * arrays each), kept for the next call with the same sizes. */
nh_status nh_adjoint_run(nh_solver *s, int64_t nsteps, int32_t ngauges,
                         const int32_t *gauges, const double *target,
                         int32_t ckpt_every, double adj_tol, double *J,
                         double *dJ_dh0, double *dJ_dhu0, double *dJ_dhv0,
                         double *dJ_dH);

/* ---- Ensembles -----------------------------------------------------------
 * n independent 2D grids ("members", e.g. scenarios of one basin or of
 * different basins) advanced together on one stream.  Each phase of a time
 * step (Section 6: two projection-correction stages and the CFL reduction,
 * eq. 23) is one launch over all members; the relaxation solves (eq. 32) of
 * all members run in lockstep cycles of sweeps, and each member leaves them at
 * its own convergence check.  A member computes exactly what a single solver
 * with its grid and parameters computes (same kernels, same arithmetic, bit
 * for bit), with its own dt, sweep counts and status.
 *
 * Members must be 2D (ny >= 2) and share precision, nh_on, breaking_on,
 * solve_max_iter and check_every; everything else (grid, dt or CFL, dry
 * threshold, tolerance, relaxation schedule) may differ.  Arrays have the
 * layout of the single-grid calls for the member's grid.  A member whose state
 * fails (non-finite values, no wet cell) leaves the ensemble until its state
 * is set again; the others go on.
 */
typedef struct nh_ensemble nh_ensemble;

/* grids[n], params[n] (copied).  Allocates every member's device memory.
 * The members share precision, nh_on, breaking_on, solve_max_iter,
 * check_every and solve_path (NH_EINVAL otherwise). */
nh_status nh_ensemble_create(int32_t n, const nh_grid *grids,
                             const nh_params *params, void *hip_stream,
                             nh_ensemble **out);
nh_status nh_ensemble_set_bathymetry(nh_ensemble *e, int32_t member,
                                     const double *H);
/* As nh_set_state, for one member (resets its time, steps and statistics). */
nh_status nh_ensemble_set_state(nh_ensemble *e, int32_t member,
                                const double *h, const double *hu,
                                const double *hv, const double *w,
                                const double *p);
/* Sweep tile of a member, bx x by corners per workgroup, with bx, by >= 4
 * and (bx + 16)(by + 16) <= 2048 in an FP64 ensemble, <= 3072 in an FP32
 * ensemble (3 region points per thread of a 1024-thread workgroup).  The tile
 * changes only the speed, never the result.  Default: 24 x 24, or 32 x 32 for
 * an FP32 member of more than 1024 such tiles. */
nh_status nh_ensemble_set_tile(nh_ensemble *e, int32_t member, int32_t bx,
                               int32_t by);
nh_status nh_ensemble_get_tile(const nh_ensemble *e, int32_t member,
                               int32_t *bx, int32_t *by);
/* Autotuner: for every distinct grid shape, times one launch of 8 sweeps
 * for each candidate tile on a synthetic system of that shape (best of
 * `reps` after a warm-up) and gives the fastest tile to the members of that
 * shape. */
nh_status nh_ensemble_tune(nh_ensemble *e, int32_t reps);
/* nsteps steps of every member that has a valid state.  Returns NH_OK, or
 * the first status of a member that failed (the others still completed the
 * steps). */
nh_status nh_ensemble_run(nh_ensemble *e, int64_t nsteps);
/* As nh_ensemble_run, for an ensemble whose solves are one launch each
 * (solve_path 2): a step is then a fixed sequence of launches that waits for
 * nothing on the host, captured once into a HIP graph (again after the
 * members' tables change) and replayed nsteps times on the ensemble's
 * stream, with the statuses read every 64 steps.  The solves in the graph
 * are plain launches of no more workgroups than the device holds at once
 * (graphs take no cooperative launch); their waits are bounded.  Results
 * equal nh_ensemble_run's to the bit.  NH_EINVAL for other solve paths or
 * while profiling; a member that fails stops the replay at the next status
 * read. */
nh_status nh_ensemble_run_graph(nh_ensemble *e, int64_t nsteps);
nh_status nh_ensemble_read_state(nh_ensemble *e, int32_t member, double *h,
                                 double *hu, double *hv, double *w, double *p);
/* Member statistics as of the end of the last run.  last_status is the
 * member's failure status, else NH_ENOCONV if one of its solves since its
 * state was set reached solve_max_iter, else NH_OK. */
nh_status nh_ensemble_get_stats(const nh_ensemble *e, int32_t member,
                                nh_stats *out);
/* Per-phase timing summed over all members (modes as nh_profile). */
nh_status nh_ensemble_profile(nh_ensemble *e, int32_t on);
nh_status nh_ensemble_get_profile(nh_ensemble *e, nh_profile_t *out);
void nh_ensemble_destroy(nh_ensemble *e);

/* ---- Without allocation --------------------------------------------------
 * For callers that cannot allocate device memory: tight serving loops,
 * harnesses that forbid hipMalloc.  (Stream capture is not supported: each
 * relaxation cycle reads its convergence measure back to the host.)
 *
 * nh_run_noalloc runs nsteps time steps as nh_create + nh_bind_device_buffers
 * + nh_run + nh_read_state would, on the same kernels and with the same
 * results bit for bit, without a solver object: the bathymetry H and the
 * state U^n = (h, hu, hv) and w are caller-owned device buffers of the
 * solver's device (the current HIP device), element type of the precision
 * (double for NH_FP64, float for NH_FP32), contiguous, row-major: H, h, hu,
 * hv cells [ny][nx] (hv ignored in 1D, may be NULL), w corners [ny+1][nx+1]
 * ([nx+1] in 1D); in NH_FP32 the h buffer holds s = h - max(H, 0) (the
 * depth storage of nh_device_views).  p: FP64 device array over the corners, the
 * warm start of the first solve on entry (zeros for none) and the last
 * solve's pressure on return.  h, hu, hv, w and p are updated in place; H is only read.  Every
 * other array (stage states, the pressure system, the relaxation iterates,
 * reductions, dt, statistics) is carved from one static device array of
 * NH_NOALLOC_SCRATCH_BYTES that each device holds from the library's load
 * until the process ends: the call makes no hipMalloc, hipHostMalloc or
 * hipFree.  A grid whose arrays do not fit (about 128 B per cell in FP64,
 * 64 B in FP32, more with breaking; a 512 x 512 FP64 grid fits) gets
 * NH_EINVAL.  The scratch is cleared at the start of every call, so no call
 * depends on the one before; calls that overlap on one device (other
 * threads, other streams) share it and race.  Relaxation zones are not
 * available; the solves are launches of 8 sweeps (solve_path 2 gets
 * NH_EINVAL).  stats (host, nullable) receives the run's statistics (t from
 * 0).  Errors as nh_run, and NH_EINVAL / NH_ENEGDEPTH for non-finite values
 * or h < 0 in the buffers (checked on the device).  Synchronises hip_stream
 * (NULL: the null stream). */
#define NH_NOALLOC_SCRATCH_BYTES (64u << 20)
nh_status nh_run_noalloc(const nh_grid *grid, const nh_params *params,
                         void *hip_stream, const void *H, void *h, void *hu,
                         void *hv, void *w, double *p, int64_t nsteps,
                         nh_stats *stats);

/* Thread-local message of the last failing call ("" if none). */
const char *nh_last_error(void);

/* Library version string. */
const char *nh_version(void);

#ifdef __cplusplus
}
#endif
#endif /* NHSWE_H */
