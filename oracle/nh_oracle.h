/*
 * nh_oracle.h -- plain FP64 CPU oracle of the projection-correction scheme for
 * the depth-integrated non-hydrostatic (Yamazaki) shallow-water system of
 * Escalante, Morales de Luna & Castro, "Non-Hydrostatic Pressure Shallow
 * Flows: GPU Implementation Using Finite Volume and Finite Difference Scheme"
 * (arXiv 1706.04551).
 *
 * TEST INFRASTRUCTURE. This oracle exists to check the GPU library. Only the
 * test-suite, the smoke check and the benchmark's CPU-baseline leg may load
 * it. It shares no source, header, table or helper with the GPU library.
 *
 * Array conventions of this interface (all host memory, caller-owned, FP64):
 *   cells   : [ny][nx], x fastest.  In 1D mode (ny == 1) simply [nx].
 *   corners : [ny+1][nx+1] in 2D, [nx+1] in 1D.  Corner (k, l) sits at
 *             x = k*dx, y = l*dy; cell (i, j) has corners (i,j) SW, (i+1,j) SE,
 *             (i,j+1) NW, (i+1,j+1) NE.
 * Walls on every side unless open (outflow) or periodic (mirror ghosts at
 * walls: the state is even, the normal discharge odd).
 */
#ifndef NH_ORACLE_H
#define NH_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ora_params {
  int32_t nx, ny;          /* ny == 1 selects the 1D channel of Section 4 */
  double dx, dy;
  double g, cfl;
  double delta;            /* desingularisation depth of Section 4.5 */
  double dry_eps;          /* h <= dry_eps is a dry cell */
  int32_t nh_on;           /* 0: hydrostatic SWE only (no pressure step) */
  int32_t breaking_on;     /* eddy-viscosity breaking terms of Section 3 */
  double b1, b2;           /* breaking calibration coefficients, eq. (9) */
  int32_t solve_max_iter;  /* cap on relaxation sweeps (2D) */
  int32_t check_every;     /* convergence test every this many sweeps */
  double solve_tol;        /* stop when max |D^-1 (rhs - A p)| < solve_tol */
  int32_t fixed_dt;        /* 1: use dt_fixed for every step */
  double dt_fixed;
  double manning;          /* Gauckler-Manning n of the friction law of
                              Section 2 [s m^-1/3]; 0: no friction */
  int32_t open_sides;      /* outflow sides of Section 4.4 (homogeneous
                              Neumann ghosts), a bit each: 1 west, 2 east,
                              4 south, 8 north; the others are walls */
  int32_t periodic;        /* periodic directions of Section 4.4, item 1:
                              1 x, 2 y (ignored in 1D).  The first and last
                              cells of a periodic line are neighbours; its
                              last corner is its first (both are kept and
                              hold the same values) */
  int32_t w_advection;     /* 0: the vertical velocity equation of the model,
                              h w_t = p (eq. 7); 1: the energy-consistent
                              form (hw)_t + div(hw u) = p named after eq. 7,
                              i.e. h (w_t + u . grad w) = p: w is carried by
                              the flow in each stage's hyperbolic step */
  int32_t solve_norm;      /* stop measure of the relaxation (2D): 0 the size
                              of a plain Jacobi update, max |(rhs - A p) /
                              diag| (eq. 32); 1 the relative residual
                              max |rhs - A p| / max |rhs| (the absolute one
                              when rhs = 0) */
} ora_params;

/* status codes */
enum { ORA_OK = 0, ORA_EINVAL = -1, ORA_ENOCONV = -4, ORA_ENONFINITE = -5,
       ORA_ENEGDEPTH = -6, ORA_ENODOM = -7 };

typedef struct ora ora_t;

ora_t *ora_create(const ora_params *p, const double *omega, int32_t n_omega);
void ora_destroy(ora_t *o);
int ora_set_bathymetry(ora_t *o, const double *H);
int ora_set_state(ora_t *o, const double *h, const double *q1, const double *q2,
                  const double *w, const double *p);
int ora_get_state(const ora_t *o, double *h, double *q1, double *q2, double *w,
                  double *p);
/* One full RK2 step (Section 4.3 / Appendix A, TVD-RK2). Returns a status. */
int ora_step(ora_t *o);
int ora_run(ora_t *o, int64_t nsteps);
/* stats[0]=t, [1]=dt of the next step, [2]=steps taken, [3]=sweeps stage 1
 * of the last step, [4]=sweeps stage 2, [5]=last convergence measure,
 * [6]=clamped mass (total), [7]=total sweeps, [8]=total solves,
 * [9]=dt used by the last step, [10]=last status, [11]=corners of the last
 * step whose pressure row was not strictly diagonally dominant */
void ora_get_stats(const ora_t *o, double *stats);

/* ---- component entry points (used by the pinning tests) ---- */
/* CFL time step (eq. 23; 2D sum form) of a cell state. */
double ora_cfl_dt(ora_t *o, const double *h, const double *q1,
                  const double *q2);
/* Finite-volume stage U* = V - dt*(...) (eqs. 18-22, 30) + positivity.
 * Returns the clamped mass through *clamped (nullable). */
int ora_fv_stage(ora_t *o, const double *h, const double *q1, const double *q2,
                 double dt, double *h_out, double *q1_out, double *q2_out,
                 double *clamped);
/* Breaking terms (Section 3, eqs. 9-12, 28): q += dt*R_u, w += dt*R_w/h_c. */
/* Generation/absorption zones of Section 4.4.  widths[4] = L of the west,
 * east, south, north walls [m] (0: none; south/north ignored in 1D).
 * Targets: h_t, q1_t, q2_t over the cells (row-major ny x nx), w_t, p_t over
 * the corners; NULL gives still water (h* = max(H, 0), q* = w* = p* = 0).
 * Call after ora_set_bathymetry.  All widths 0 switches the zones off. */
int ora_set_relaxation(ora_t *o, const double *widths, const double *h_t,
                       const double *q1_t, const double *q2_t,
                       const double *w_t, const double *p_t);
int ora_breaking(ora_t *o, const double *h, double *q1, double *q2, double *w,
                 double dt);
/* Pressure system coefficients.  2D: 5-point closed form, rows scaled as
 * A p = rhs with diag entry 16 + ...; 1D: eq. (43) a (west), b (diag), c (east)
 * and the right-hand side, rows scaled by dx^2.  Wall rows are folded. */
int ora_assemble(ora_t *o, const double *h, const double *q1, const double *q2,
                 const double *w, double dt, double *diag, double *cE,
                 double *cW, double *cN, double *cS, double *rhs);
/* Literal discrete constraint B at every corner: eq. (37) with the edge
 * values of the final scheme (2D), eq. (24)-(25) (1D), after the correction
 * by p. */
int ora_constraint(ora_t *o, const double *h, const double *q1,
                   const double *q2, const double *w, const double *p,
                   double dt, double *out);
/* Solve A p = rhs: Thomas (1D) or relaxed Jacobi with the schedule (2D).
 * p is the warm start on entry. */
int ora_solve(ora_t *o, const double *diag, const double *cE, const double *cW,
              const double *cN, const double *cS, const double *rhs, double *p,
              int32_t *sweeps, double *measure);
/* Dense Gaussian elimination with partial pivoting of the same system
 * (validation only; corners <= 4096). */
int ora_dense_solve(ora_t *o, const double *diag, const double *cE,
                    const double *cW, const double *cN, const double *cS,
                    const double *rhs, double *p);
/* Correction (eq. 36 / eq. 26-28): q += dt*T_NH, w += dt*p/h_c. */
int ora_correct(ora_t *o, const double *h, const double *q1, const double *q2,
                const double *w, const double *p, double dt, double *q1_out,
                double *q2_out, double *w_out);
/* One edge fluctuation, eq. (18)-(19) with the wet-dry rule.
 * left/right = {h, qn, qt, un, ut, eta, H}; Dm/Dp = 3 components. */
void ora_pvm_fluct(const double *left, const double *right, double g,
                   double dry_eps, double *Dm, double *Dp);
/* The desingularised velocity of Section 4.5. */
double ora_desing_velocity(double h, double q, double delta);

#ifdef __cplusplus
}
#endif
#endif
