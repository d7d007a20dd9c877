/*
 * nh_oracle.c -- plain, slow, FP64 CPU oracle of the projection-correction
 * scheme of Escalante, Morales de Luna & Castro (arXiv 1706.04551).
 *
 * TEST INFRASTRUCTURE: this file is the reference the GPU library is checked
 * against.  It is loaded only by the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg, and it shares no code with the GPU library.
 * Compile with -O2 -ffp-contract=off and no fast-math.
 *
 * The code follows the paper step by step:
 *   Section 4.1  finite-volume PVM step, eqs. (16)-(22)
 *   Section 4.2  staggered finite differences, eqs. (24)-(27)
 *   Section 4.3  projection system, eq. (28)-(29); Appendix "A.1" eq. (42)-(43)
 *   Section 4.5  wet-dry treatment and the desingularised velocity
 *   Section 5 / Appendix A  the 2D scheme, eqs. (30)-(41)
 *   Section 3    breaking terms, eqs. (9)-(12)
 * Where the paper is silent or garbled, the readings used are listed in the
 * repository's design notes; the ones that shape code are restated inline.
 *
 * Pins: every function below is checked by the CPU tests against closed
 * forms, invariants or brute force (lake at rest, mass, dispersion relation,
 * eq. (43), the small-depth closed form, probe assembly of the matrix from the
 * literal constraint, dense solves, Thomas, y-invariance, mirror symmetry).
 */
#include "nh_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define GH 2 /* ghost layers: MUSCL needs the neighbour's slope */

struct ora {
  ora_params P;
  int is1d;
  int nx, ny;   /* interior cells */
  int gx, gy;   /* ghosted dims */
  int goy;      /* ghost offset in y (0 in 1D) */
  int ncx, ncy; /* corner dims */
  double *omega;
  int n_omega;
  /* persistent state, ghosted cells + corners */
  double *H, *h, *q1, *q2;
  double *w, *p;
  double dt, t, dt_last;
  long step;
  long sweeps_stage[2];
  double measure_last;
  double clamped_total;
  long sweeps_total, solves_total;
  long nondom_last; /* corners whose row was not strictly dominant */
  int last_status;
  /* work buffers */
  double *b[16];  /* ghosted cell buffers */
  double *c[16];  /* corner buffers */
  /* relaxation zones (Section 4.4): weights and targets, NULL when off */
  double *rm_cell, *rm_corn;               /* m of cells (ghosted), corners */
  double *rt_h, *rt_q1, *rt_q2, *rt_w, *rt_p;
};

/* ------------------------------------------------------------------ */
/* indexing                                                           */
/* ------------------------------------------------------------------ */
static inline int IX(const ora_t *o, int i, int j) {
  return (j + o->goy) * o->gx + (i + GH);
}
static inline int CX(const ora_t *o, int k, int l) { return l * o->ncx + k; }
/* Corner reflection about a wall corner row (reading: mirror ghosts also for
 * the corner unknowns, so that p_{-1} = p_{1}); in a periodic direction the
 * corners wrap around (corner n is corner 0, so k < 0 is k + n and k > n is
 * k - n). */
static inline int refl(int k, int n, int per) {
  if (per) return k < 0 ? k + n : (k > n ? k - n : k);
  if (k < 0) return -k;
  if (k > n) return 2 * n - k;
  return k;
}
static inline int per_x(const ora_t *o) { return o->P.periodic & 1; }
static inline int per_y(const ora_t *o) {
  return !o->is1d && (o->P.periodic & 2);
}
static inline double P_at(const ora_t *o, const double *p, int k, int l) {
  return p[CX(o, refl(k, o->nx, per_x(o)),
              o->is1d ? 0 : refl(l, o->ny, per_y(o)))];
}

static double dmax(double a, double b) { return a > b ? a : b; }
static double dmin(double a, double b) { return a < b ? a : b; }

/* minmod limiter used by the MUSCL reconstruction (Section 4.1) */
static double minmod(double a, double b) {
  if (a > 0.0 && b > 0.0) return dmin(a, b);
  if (a < 0.0 && b < 0.0) return dmax(a, b);
  return 0.0;
}

/* Desingularised velocity, Section 4.5:
 *   u = sqrt(2) h q / sqrt(h^4 + max(h^4, delta^4)). */
double ora_desing_velocity(double h, double q, double delta) {
  double h4 = h * h * h * h;
  double d4 = delta * delta * delta * delta;
  return sqrt(2.0) * h * q / sqrt(h4 + dmax(h4, d4));
}
/* Same desingularised division used for w = w* + dt p / h_c at corners
 * (reading: the corner update divides by h_c the way velocities do, so that a
 * dry corner keeps its w). */
static double desing_div(double num, double h, double delta) {
  return ora_desing_velocity(h, num, delta);
}

/* Mirror ghosts on walls (walls are the only boundary on the hot path):
 * ghost -1 <-> cell 0, ghost -2 <-> cell 1, and likewise on the far side.
 * px / py = +1 (even) or -1 (odd) parity across x / y walls. */
static void fill_ghosts(const ora_t *o, double *a, double px, double py) {
  /* Outflow sides (Section 4.4, homogeneous Neumann): the ghosts take the
   * value of the adjacent cell, with no change of sign.  Periodic
   * directions (Section 4.4, item 1): the first and last cells of a line are
   * neighbours, so the ghosts past one end are the cells at the other end,
   * with no change of sign. */
  const int open = o->P.open_sides;
  const int px_per = per_x(o), py_per = per_y(o);
  int nx = o->nx, ny = o->ny;
  for (int j = 0; j < ny; ++j)
    for (int g = 1; g <= GH; ++g) {
      if (px_per) {
        a[IX(o, -g, j)] = a[IX(o, nx - g, j)];
        a[IX(o, nx - 1 + g, j)] = a[IX(o, g - 1, j)];
        continue;
      }
      a[IX(o, -g, j)] = (open & 1) ? a[IX(o, 0, j)] : px * a[IX(o, g - 1, j)];
      a[IX(o, nx - 1 + g, j)] =
          (open & 2) ? a[IX(o, nx - 1, j)] : px * a[IX(o, nx - g, j)];
    }
  if (o->is1d) return;
  for (int i = -GH; i < nx + GH; ++i)
    for (int g = 1; g <= GH; ++g) {
      if (py_per) {
        a[IX(o, i, -g)] = a[IX(o, i, ny - g)];
        a[IX(o, i, ny - 1 + g)] = a[IX(o, i, g - 1)];
        continue;
      }
      a[IX(o, i, -g)] = (open & 4) ? a[IX(o, i, 0)] : py * a[IX(o, i, g - 1)];
      a[IX(o, i, ny - 1 + g)] =
          (open & 8) ? a[IX(o, i, ny - 1)] : py * a[IX(o, i, ny - g)];
    }
}

static void load_cells(const ora_t *o, double *dst, const double *src) {
  for (int j = 0; j < o->ny; ++j)
    for (int i = 0; i < o->nx; ++i) dst[IX(o, i, j)] = src[j * o->nx + i];
}
static void store_cells(const ora_t *o, double *dst, const double *src) {
  for (int j = 0; j < o->ny; ++j)
    for (int i = 0; i < o->nx; ++i) dst[j * o->nx + i] = src[IX(o, i, j)];
}
static int ncorners(const ora_t *o) { return o->ncx * o->ncy; }

/* ------------------------------------------------------------------ */
/* Section 4.1: PVM path-conservative fluctuations                     */
/* ------------------------------------------------------------------ */
typedef struct {
  double h, qn, qt, un, ut, eta, H;
} face_t;

/*
 * First-order PVM fluctuation of eq. (18)-(19) between a left state L and a
 * right state R (reconstructed states of eq. (21) in the second-order scheme),
 * with the A* replacement of the Roe matrix, Q = alpha0 Id + alpha1 A, the HLL
 * speeds S_L, S_R and the Roe average of Section 4.1.
 *   D+- = 1/2 [ (1 +- alpha1) R +- alpha0 (dEta, dqn, dqt) ]
 *   R   = ( dqn, d(qn un) + g h_e dEta, d(qn ut) )
 * In 2D (Section 5) the same expression is applied normal to each edge, the
 * tangential discharge being carried with the same alpha0, alpha1.
 * Wet-dry rule for emerging bottoms (Section 4.5): when one side is dry and
 * its bed lies above the free surface of the wet side, the surface jump seen
 * by the hydrostatic pressure term is set to zero (the dry bed acts as a wall
 * for the pressure force).  Both sides dry: no fluctuation.
 */
static void pvm_fluct(const face_t *L, const face_t *R, double g,
                      double dry_eps, double Dm[3], double Dp[3]) {
  Dm[0] = Dm[1] = Dm[2] = 0.0;
  Dp[0] = Dp[1] = Dp[2] = 0.0;
  if (L->h <= dry_eps && R->h <= dry_eps) return;
  double he = 0.5 * (L->h + R->h);
  double sL = sqrt(L->h), sR = sqrt(R->h);
  double ue = (L->un * sL + R->un * sR) / (sL + sR);
  double ce = sqrt(g * he);
  double SL = dmin(ue - ce, L->un - sqrt(g * L->h));
  double SR = dmax(ue + ce, R->un + sqrt(g * R->h));
  if (!(SR - SL > 0.0)) return;
  double a0 = (SR * fabs(SL) - SL * fabs(SR)) / (SR - SL);
  double a1 = (fabs(SR) - fabs(SL)) / (SR - SL);
  double deta = R->eta - L->eta;
  if (R->h <= dry_eps && L->eta < -R->H) deta = 0.0;
  if (L->h <= dry_eps && R->eta < -L->H) deta = 0.0;
  double Rv[3], dU[3];
  Rv[0] = R->qn - L->qn;
  Rv[1] = (R->qn * R->un - L->qn * L->un) + g * he * deta;
  Rv[2] = R->qn * R->ut - L->qn * L->ut;
  dU[0] = deta;
  dU[1] = R->qn - L->qn;
  dU[2] = R->qt - L->qt;
  for (int m = 0; m < 3; ++m) {
    Dm[m] = 0.5 * ((1.0 - a1) * Rv[m] - a0 * dU[m]);
    Dp[m] = 0.5 * ((1.0 + a1) * Rv[m] + a0 * dU[m]);
  }
}

void ora_pvm_fluct(const double *left, const double *right, double g,
                   double dry_eps, double *Dm, double *Dp) {
  face_t L = {left[0], left[1], left[2], left[3], left[4], left[5], left[6]};
  face_t R = {right[0], right[1], right[2], right[3], right[4], right[5],
              right[6]};
  pvm_fluct(&L, &R, g, dry_eps, Dm, Dp);
}

/*
 * MUSCL reconstruction with the minmod limiter along one direction (Section
 * 4.1): h, eta and the velocities are reconstructed; q = h u and H = h - eta
 * are recovered from them.  The slopes of eta and of the velocities are set
 * to zero in a cell with a dry neighbour (or dry itself), so that emerging
 * topography creates no spurious pressure gradient.
 * Outputs: Lf = value at the cell's minus-side edge (U^+_{i-1/2}),
 *          Rf = value at the cell's plus-side edge  (U^-_{i+1/2}).
 */
static void reconstruct(double hm, double h0, double hp, double em, double e0,
                        double ep, double um, double u0, double up, double vm,
                        double v0, double vp, double dry_eps, face_t *Lf,
                        face_t *Rf) {
  double sh = minmod(hp - h0, h0 - hm);
  double se = 0.0, su = 0.0, sv = 0.0;
  if (hm > dry_eps && h0 > dry_eps && hp > dry_eps) {
    se = minmod(ep - e0, e0 - em);
    su = minmod(up - u0, u0 - um);
    sv = minmod(vp - v0, v0 - vm);
  }
  Rf->h = h0 + 0.5 * sh;
  Lf->h = h0 - 0.5 * sh;
  Rf->eta = e0 + 0.5 * se;
  Lf->eta = e0 - 0.5 * se;
  Rf->un = u0 + 0.5 * su;
  Lf->un = u0 - 0.5 * su;
  Rf->ut = v0 + 0.5 * sv;
  Lf->ut = v0 - 0.5 * sv;
  Rf->qn = Rf->h * Rf->un;
  Lf->qn = Lf->h * Lf->un;
  Rf->qt = Rf->h * Rf->ut;
  Lf->qt = Lf->h * Lf->ut;
  Rf->H = Rf->h - Rf->eta;
  Lf->H = Lf->h - Lf->eta;
}

/*
 * Volume term I_i of eq. (22) for one direction, written as
 *   ( qn^- - qn^+,  qn^- un^- - qn^+ un^+ + g h_i (eta^- - eta^+),
 *     qn^- ut^- - qn^+ ut^+ )
 * where ^- is the value at the plus-side edge (U^-_{i+1/2}) and ^+ at the
 * minus-side edge (U^+_{i-1/2}).  The hydrostatic part of eq. (22),
 * 1/2 g (h^-^2 - h^+^2) - g h_i (H^- - H^+), equals g h_i (eta^- - eta^+)
 * because the linear reconstruction has h^- + h^+ = 2 h_i; this is also the
 * mid-point rule of the volume integral in eq. (30).  In this form the lake
 * at rest is preserved exactly in floating point.
 */
static void interior_term(const face_t *Lf, const face_t *Rf, double h0,
                          double g, double I[3]) {
  I[0] = Rf->qn - Lf->qn;
  I[1] = (Rf->qn * Rf->un - Lf->qn * Lf->un) + g * h0 * (Rf->eta - Lf->eta);
  I[2] = Rf->qn * Rf->ut - Lf->qn * Lf->ut;
}

/* ------------------------------------------------------------------ */
/* finite-volume stage on ghosted arrays                                */
/* ------------------------------------------------------------------ */
/* Vh,Vq1,Vq2 ghosted with ghosts filled; outputs interior only. */
static void fv_stage_g(ora_t *o, const double *Vh, const double *Vq1,
                       const double *Vq2, double dt, double *Oh, double *Oq1,
                       double *Oq2, double *clamped) {
  const double g = o->P.g, de = o->P.delta, eps = o->P.dry_eps;
  const int nx = o->nx, ny = o->ny;
  const int N = o->gx * o->gy;
  double *u = o->b[8], *v = o->b[9], *eta = o->b[10];
  for (int n = 0; n < N; ++n) {
    u[n] = ora_desing_velocity(Vh[n], Vq1[n], de);
    v[n] = o->is1d ? 0.0 : ora_desing_velocity(Vh[n], Vq2[n], de);
    eta[n] = Vh[n] - o->H[n];
  }
  /* faces of every cell in x, for i in [-1, nx], j in [0, ny) */
  int nfx = (nx + 2) * ny;
  face_t *xL = (face_t *)malloc(sizeof(face_t) * nfx);
  face_t *xR = (face_t *)malloc(sizeof(face_t) * nfx);
#define FXI(i, j) ((j) * (nx + 2) + (i) + 1)
  for (int j = 0; j < ny; ++j)
    for (int i = -1; i <= nx; ++i) {
      int c = IX(o, i, j), m = IX(o, i - 1, j), p = IX(o, i + 1, j);
      reconstruct(Vh[m], Vh[c], Vh[p], eta[m], eta[c], eta[p], u[m], u[c],
                  u[p], v[m], v[c], v[p], eps, &xL[FXI(i, j)], &xR[FXI(i, j)]);
    }
  face_t *yL = NULL, *yR = NULL;
  int nfy = nx * (ny + 2);
#define FYI(i, j) (((j) + 1) * nx + (i))
  if (!o->is1d) {
    yL = (face_t *)malloc(sizeof(face_t) * nfy);
    yR = (face_t *)malloc(sizeof(face_t) * nfy);
    for (int j = -1; j <= ny; ++j)
      for (int i = 0; i < nx; ++i) {
        int c = IX(o, i, j), m = IX(o, i, j - 1), p = IX(o, i, j + 1);
        /* normal = y: normal velocity v, tangential u */
        reconstruct(Vh[m], Vh[c], Vh[p], eta[m], eta[c], eta[p], v[m], v[c],
                    v[p], u[m], u[c], u[p], eps, &yL[FYI(i, j)],
                    &yR[FYI(i, j)]);
      }
  }
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      int c = IX(o, i, j);
      double Dm_e[3], Dp_e[3], Dm_w[3], Dp_w[3], I[3];
      /* x: edge i+1/2 between cell i (its plus face) and i+1 (its minus face)
       */
      pvm_fluct(&xR[FXI(i, j)], &xL[FXI(i + 1, j)], g, eps, Dm_e, Dp_e);
      pvm_fluct(&xR[FXI(i - 1, j)], &xL[FXI(i, j)], g, eps, Dm_w, Dp_w);
      interior_term(&xL[FXI(i, j)], &xR[FXI(i, j)], Vh[c], g, I);
      double fx[3];
      for (int m = 0; m < 3; ++m) fx[m] = (Dm_e[m] + Dp_w[m]) + I[m];
      double fy[3] = {0.0, 0.0, 0.0};
      if (!o->is1d) {
        double Dm_n[3], Dp_n[3], Dm_s[3], Dp_s[3], J[3];
        pvm_fluct(&yR[FYI(i, j)], &yL[FYI(i, j + 1)], g, eps, Dm_n, Dp_n);
        pvm_fluct(&yR[FYI(i, j - 1)], &yL[FYI(i, j)], g, eps, Dm_s, Dp_s);
        interior_term(&yL[FYI(i, j)], &yR[FYI(i, j)], Vh[c], g, J);
        for (int m = 0; m < 3; ++m) fy[m] = (Dm_n[m] + Dp_s[m]) + J[m];
      }
      /* x components are (h, q1, q2); y components are (h, q2, q1) */
      double hs, q1s, q2s;
      if (o->is1d) {
        hs = Vh[c] - dt * (fx[0] / o->P.dx);
        q1s = Vq1[c] - dt * (fx[1] / o->P.dx);
        q2s = 0.0;
      } else {
        hs = Vh[c] - dt * (fx[0] / o->P.dx + fy[0] / o->P.dy);
        q1s = Vq1[c] - dt * (fx[1] / o->P.dx + fy[2] / o->P.dy);
        q2s = Vq2[c] - dt * (fx[2] / o->P.dx + fy[1] / o->P.dy);
      }
      /* positivity: negative depth is clamped (and counted); a dry cell
       * carries no discharge */
      if (hs < 0.0) {
        if (clamped) *clamped += -hs * o->P.dx * (o->is1d ? 1.0 : o->P.dy);
        hs = 0.0;
      }
      if (hs <= eps) {
        q1s = 0.0;
        q2s = 0.0;
      }
      Oh[c] = hs;
      Oq1[c] = q1s;
      Oq2[c] = q2s;
    }
  free(xL);
  free(xR);
  free(yL);
  free(yR);
#undef FXI
#undef FYI
}

/* CFL condition (eq. 23); in 2D the x and y wave-speed ratios are added
 * (reading): dt = CFL / max((|u|+c)/dx + (|v|+c)/dy) over wet cells. */
static double cfl_dt_g(const ora_t *o, const double *h, const double *q1,
                       const double *q2) {
  double lam = 0.0;
  for (int j = 0; j < o->ny; ++j)
    for (int i = 0; i < o->nx; ++i) {
      int c = IX(o, i, j);
      if (!(h[c] > o->P.dry_eps)) continue;
      double cel = sqrt(o->P.g * h[c]);
      double u = ora_desing_velocity(h[c], q1[c], o->P.delta);
      double l = (fabs(u) + cel) / o->P.dx;
      if (!o->is1d) {
        double v = ora_desing_velocity(h[c], q2[c], o->P.delta);
        l = l + (fabs(v) + cel) / o->P.dy;
      }
      if (l > lam) lam = l;
    }
  if (!(lam > 0.0)) return 0.0;
  return o->P.cfl / lam;
}

/* ------------------------------------------------------------------ */
/* Section 3: breaking terms                                            */
/* ------------------------------------------------------------------ */
/*
 * Eddy viscosity nu = max(0, B) h |q_x|, B = 1 - q_x / U1, U1 = B1 sqrt(g h)
 * (eq. 9; nu = 0 where B < 0).  In 2D q_x and u_x become div q and div u
 * (reading of Section 5: "following the ideas of Section 3").  The parabolic
 * term is moved into the pressure (eqs. 10-12), leaving the explicit terms
 *   R_u = 2 nu (div u) grad H   in the momentum equation,
 *   R_w = 2 nu (div u)          in h w_t = p + R_w,
 * with centred differences at cells (Section 4.3).  R_w is averaged from the
 * cells to the corner and divided by h_c there.  h, q ghosted and filled;
 * q updated in place (interior), w (corners) updated in place.
 */
static void breaking_g(ora_t *o, const double *h, double *q1, double *q2,
                       double *w, double dt) {
  const double g = o->P.g, de = o->P.delta, eps = o->P.dry_eps;
  const int nx = o->nx, ny = o->ny;
  const double dx = o->P.dx, dy = o->P.dy;
  double *rw = o->b[11], *u = o->b[8], *v = o->b[9];
  int N = o->gx * o->gy;
  for (int n = 0; n < N; ++n) {
    u[n] = ora_desing_velocity(h[n], q1[n], de);
    v[n] = o->is1d ? 0.0 : ora_desing_velocity(h[n], q2[n], de);
    rw[n] = 0.0;
  }
  int jlo = o->is1d ? 0 : -1, jhi = o->is1d ? 0 : ny;
  double *dq1 = o->b[12], *dq2 = o->b[13];
  for (int j = jlo; j <= jhi; ++j)
    for (int i = -1; i <= nx; ++i) {
      int c = IX(o, i, j);
      double divq = (q1[IX(o, i + 1, j)] - q1[IX(o, i - 1, j)]) / (2.0 * dx);
      double divu = (u[IX(o, i + 1, j)] - u[IX(o, i - 1, j)]) / (2.0 * dx);
      double Hx = (o->H[IX(o, i + 1, j)] - o->H[IX(o, i - 1, j)]) / (2.0 * dx);
      double Hy = 0.0;
      if (!o->is1d) {
        divq += (q2[IX(o, i, j + 1)] - q2[IX(o, i, j - 1)]) / (2.0 * dy);
        divu += (v[IX(o, i, j + 1)] - v[IX(o, i, j - 1)]) / (2.0 * dy);
        Hy = (o->H[IX(o, i, j + 1)] - o->H[IX(o, i, j - 1)]) / (2.0 * dy);
      }
      double nu = 0.0;
      if (h[c] > eps) {
        double U1 = o->P.b1 * sqrt(g * h[c]);
        double B = 1.0 - divq / U1;
        if (B > 0.0) nu = B * h[c] * fabs(divq);
      }
      rw[c] = 2.0 * nu * divu;
      dq1[c] = dt * rw[c] * Hx;
      dq2[c] = dt * rw[c] * Hy;
    }
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      int c = IX(o, i, j);
      q1[c] = q1[c] + dq1[c];
      if (!o->is1d) q2[c] = q2[c] + dq2[c];
    }
  fill_ghosts(o, q1, -1.0, 1.0);
  if (!o->is1d) fill_ghosts(o, q2, 1.0, -1.0);
  for (int l = 0; l < o->ncy; ++l)
    for (int k = 0; k < o->ncx; ++k) {
      double hc, rwc;
      if (o->is1d) {
        hc = 0.5 * (h[IX(o, k - 1, 0)] + h[IX(o, k, 0)]);
        rwc = 0.5 * (rw[IX(o, k - 1, 0)] + rw[IX(o, k, 0)]);
      } else {
        hc = 0.25 * (h[IX(o, k - 1, l - 1)] + h[IX(o, k, l - 1)] +
                     h[IX(o, k - 1, l)] + h[IX(o, k, l)]);
        rwc = 0.25 * (rw[IX(o, k - 1, l - 1)] + rw[IX(o, k, l - 1)] +
                      rw[IX(o, k - 1, l)] + rw[IX(o, k, l)]);
      }
      w[CX(o, k, l)] = w[CX(o, k, l)] + dt * desing_div(rwc, hc, de);
    }
}

/* ------------------------------------------------------------------ */
/* pressure system                                                      */
/* ------------------------------------------------------------------ */
/*
 * 1D coefficients, eq. (43) of the appendix, rows of (42) scaled by dx^2:
 *   a_i = (xi_i - 2h_i)(xi_{i+1/2} + 2h_{i+1/2})
 *   b_i = 16dx^2 + xi_{i+1/2}(xi_i + xi_{i+1} + 2h_i - 2h_{i+1})
 *         + 2h_{i+1/2}(xi_i - xi_{i+1} + 4h_{i+1/2})
 *   c_i = (xi_{i+1} + 2h_{i+1})(xi_{i+1/2} - 2h_{i+1/2})
 * with xi = dx (2 eta_x - h_x) from eqs. (25), (27).  Right-hand side:
 *   RHS_i = -(8 dx^2/dt)(h q_x - q (2eta - h)_x + 2 h w)_{i+1/2}
 * The sign is the one obtained by substituting the correction (28) into the
 * constraint (24); the printed right-hand side has the opposite sign (reading;
 * pinned by the dispersion test and by the probe assembly).
 * Corner k sits between cell k-1 (west) and cell k (east).
 * Wall rows: the mirror p_{-1} = p_{1} folds a into c (row 0) and c into a
 * (row N): the boundary rows, which the paper leaves to be adapted.
 */
static void assemble1d_g(const ora_t *o, const double *h, const double *q,
                         const double *w, double dt, double *a, double *b,
                         double *cc, double *rhs) {
  const double dx = o->P.dx;
  double *zeta = o->b[14];
  for (int i = -GH; i < o->nx + GH; ++i)
    zeta[IX(o, i, 0)] = h[IX(o, i, 0)] - 2.0 * o->H[IX(o, i, 0)];
  for (int k = 0; k <= o->nx; ++k) {
    int W = IX(o, k - 1, 0), E = IX(o, k, 0);
    double hW = h[W], hE = h[E];
    double hc = 0.5 * (hE + hW);
    double xiW = dx * ((zeta[IX(o, k, 0)] - zeta[IX(o, k - 2, 0)]) / (2.0 * dx));
    double xiE =
        dx * ((zeta[IX(o, k + 1, 0)] - zeta[IX(o, k - 1, 0)]) / (2.0 * dx));
    double xic = dx * ((zeta[E] - zeta[W]) / dx);
    double ai = (xiW - 2.0 * hW) * (xic + 2.0 * hc);
    double bi = 16.0 * dx * dx + xic * (xiW + xiE + 2.0 * hW - 2.0 * hE) +
                2.0 * hc * (xiW - xiE + 4.0 * hc);
    double ci = (xiE + 2.0 * hE) * (xic - 2.0 * hc);
    double qc = 0.5 * (q[E] + q[W]);
    double qxc = (q[E] - q[W]) / dx;
    double zxc = (zeta[E] - zeta[W]) / dx;
    double Bc = hc * qxc - qc * zxc + 2.0 * hc * w[k];
    double r = -(8.0 * dx * dx / dt) * Bc;
    if (k == 0 && !per_x(o)) {
      ci = ci + ai;
      ai = 0.0;
    }
    if (k == o->nx && !per_x(o)) {
      ai = ai + ci;
      ci = 0.0;
    }
    a[k] = ai;
    b[k] = bi;
    cc[k] = ci;
    rhs[k] = r;
  }
}

/*
 * 2D coefficients.  The paper does not print them; they follow from
 * substituting the half corrections of the edge discharges q_{1,E}, q_{1,W},
 * q_{2,N}, q_{2,S} (final scheme of Appendix A.2) and w = w* + dt p/h_c into
 * 2 x eq. (37) and multiplying by -4/dt.  With zeta = 2 eta - h = h - 2H,
 * X_k = (zeta_{k+x} - zeta_{k-x})/2, Y_k = (zeta_{k+y} - zeta_{k-y})/2, the
 * pair averages over the east/west/north/south cells of the corner and
 * sigma_x = zeta_E - zeta_W, sigma_y = zeta_N - zeta_S (eq. 40 read with a
 * division by dx, dy):
 *   diag = 16 + [(2hc+sx)(XW+2hW) - (2hc-sx)(XE-2hE)]/dx^2 + (y alike)
 *   cE = -(2hc-sx)(XE+2hE)/dx^2,   cW = (2hc+sx)(XW-2hW)/dx^2
 *   cN = -(2hc-sy)(YN+2hN)/dy^2,   cS = (2hc+sy)(YS-2hS)/dy^2
 *   rhs = -(4/dt) B*,  B* = [(2hc-sx) q1E - (2hc+sx) q1W]/dx
 *                          + [(2hc-sy) q2N - (2hc+sy) q2S]/dy + 4 hc w*
 * Dropping y and multiplying by dx^2 gives eq. (43) exactly.
 * Walls: the mirrored neighbour is folded into the inner coefficient.  In a
 * periodic direction nothing is folded: the neighbour past the last corner
 * is the second one (corner n is corner 0), the one before the first corner
 * is corner n - 1.
 */
static void assemble2d_g(const ora_t *o, const double *h, const double *q1,
                         const double *q2, const double *w, double dt,
                         double *diag, double *cE, double *cW, double *cN,
                         double *cS, double *rhs) {
  const int nx = o->nx, ny = o->ny;
  const double dx = o->P.dx, dy = o->P.dy;
  double *zeta = o->b[14], *X = o->b[12], *Y = o->b[13];
  int N = o->gx * o->gy;
  for (int n = 0; n < N; ++n) {
    zeta[n] = h[n] - 2.0 * o->H[n];
    X[n] = 0.0;
    Y[n] = 0.0;
  }
  for (int j = -1; j <= ny; ++j)
    for (int i = -1; i <= nx; ++i) {
      X[IX(o, i, j)] = (zeta[IX(o, i + 1, j)] - zeta[IX(o, i - 1, j)]) / 2.0;
      Y[IX(o, i, j)] = (zeta[IX(o, i, j + 1)] - zeta[IX(o, i, j - 1)]) / 2.0;
    }
  for (int l = 0; l <= ny; ++l)
    for (int k = 0; k <= nx; ++k) {
      int SW = IX(o, k - 1, l - 1), SE = IX(o, k, l - 1);
      int NW = IX(o, k - 1, l), NE = IX(o, k, l);
      double hc = 0.25 * (h[SW] + h[SE] + h[NW] + h[NE]);
      double hE = 0.5 * (h[SE] + h[NE]), hW = 0.5 * (h[SW] + h[NW]);
      double hN = 0.5 * (h[NW] + h[NE]), hS = 0.5 * (h[SW] + h[SE]);
      double XE = 0.5 * (X[SE] + X[NE]), XW = 0.5 * (X[SW] + X[NW]);
      double YN = 0.5 * (Y[NW] + Y[NE]), YS = 0.5 * (Y[SW] + Y[SE]);
      double sx = 0.5 * (zeta[SE] + zeta[NE]) - 0.5 * (zeta[SW] + zeta[NW]);
      double sy = 0.5 * (zeta[NW] + zeta[NE]) - 0.5 * (zeta[SW] + zeta[SE]);
      double q1E = 0.5 * (q1[SE] + q1[NE]), q1W = 0.5 * (q1[SW] + q1[NW]);
      double q2N = 0.5 * (q2[NW] + q2[NE]), q2S = 0.5 * (q2[SW] + q2[SE]);
      double dx2 = dx * dx, dy2 = dy * dy;
      double d = 16.0 +
                 ((2.0 * hc + sx) * (XW + 2.0 * hW) -
                  (2.0 * hc - sx) * (XE - 2.0 * hE)) / dx2 +
                 ((2.0 * hc + sy) * (YS + 2.0 * hS) -
                  (2.0 * hc - sy) * (YN - 2.0 * hN)) / dy2;
      double e = -(2.0 * hc - sx) * (XE + 2.0 * hE) / dx2;
      double wv = (2.0 * hc + sx) * (XW - 2.0 * hW) / dx2;
      double n = -(2.0 * hc - sy) * (YN + 2.0 * hN) / dy2;
      double s = (2.0 * hc + sy) * (YS - 2.0 * hS) / dy2;
      double Bs = ((2.0 * hc - sx) * q1E - (2.0 * hc + sx) * q1W) / dx +
                  ((2.0 * hc - sy) * q2N - (2.0 * hc + sy) * q2S) / dy +
                  4.0 * hc * w[CX(o, k, l)];
      double r = -(4.0 / dt) * Bs;
      if (!per_x(o)) {
        if (k == 0) { e = e + wv; wv = 0.0; }
        if (k == nx) { wv = wv + e; e = 0.0; }
      }
      if (!per_y(o)) {
        if (l == 0) { n = n + s; s = 0.0; }
        if (l == ny) { s = s + n; n = 0.0; }
      }
      int c = CX(o, k, l);
      diag[c] = d;
      cE[c] = e;
      cW[c] = wv;
      cN[c] = n;
      cS[c] = s;
      rhs[c] = r;
    }
}

/* Thomas algorithm for the tridiagonal system (42) (Section 4.3). */
static int thomas(int n, const double *a, const double *b, const double *c,
                  const double *d, double *x, double *cp, double *dp) {
  if (!(b[0] != 0.0)) return ORA_ENODOM;
  cp[0] = c[0] / b[0];
  dp[0] = d[0] / b[0];
  for (int k = 1; k < n; ++k) {
    double m = b[k] - a[k] * cp[k - 1];
    if (!(m != 0.0)) return ORA_ENODOM;
    cp[k] = c[k] / m;
    dp[k] = (d[k] - a[k] * dp[k - 1]) / m;
  }
  x[n - 1] = dp[n - 1];
  for (int k = n - 2; k >= 0; --k) x[k] = dp[k] - cp[k] * x[k + 1];
  return ORA_OK;
}

/* Periodic 1D channel (Section 4.4, item 1): the rows of the nx distinct
 * corners form a cyclic tridiagonal system, row 0 reaching corner nx - 1
 * through a[0] and row nx - 1 reaching corner 0 through c[nx - 1].  The
 * "modification of the Thomas algorithm" taken here is the Sherman-Morrison
 * form: the cyclic matrix is a tridiagonal one plus the rank-one term
 * u v^T with u = (gamma, 0, ..., 0, c[n-1]), v = (1, 0, ..., 0,
 * a[0]/gamma), gamma = -b[0]; two Thomas solves with the modified diagonal
 * (b[0] - gamma, ..., b[n-1] - c[n-1] a[0] / gamma) and one correction.
 * bb, z: n work values each; cp, dp those of thomas. */
static int thomas_cyclic(int n, const double *a, const double *b,
                         const double *c, const double *d, double *x,
                         double *bb, double *z, double *cp, double *dp) {
  const double alpha = c[n - 1], beta = a[0], gamma = -b[0];
  if (!(gamma != 0.0)) return ORA_ENODOM;
  for (int k = 0; k < n; ++k) bb[k] = b[k];
  bb[0] = b[0] - gamma;
  bb[n - 1] = b[n - 1] - alpha * beta / gamma;
  int st = thomas(n, a, bb, c, d, x, cp, dp);
  if (st != ORA_OK) return st;
  /* z first holds the right-hand side u (thomas reads its right-hand side
   * before it writes the solution) */
  for (int k = 0; k < n; ++k) z[k] = 0.0;
  z[0] = gamma;
  z[n - 1] = alpha;
  st = thomas(n, a, bb, c, z, z, cp, dp);
  if (st != ORA_OK) return st;
  const double den = 1.0 + z[0] + beta * z[n - 1] / gamma;
  if (!(den != 0.0)) return ORA_ENODOM;
  const double fact = (x[0] + beta * x[n - 1] / gamma) / den;
  for (int k = 0; k < n; ++k) x[k] = x[k] - fact * z[k];
  return ORA_OK;
}

/*
 * Relaxed Jacobi with a scheduled relaxation factor (Section 5, the
 * "Jacobi method combined with a scheduled relaxation"): sweep k replaces
 *   p <- p + omega_{k mod m} (rhs - A p) / diag
 * with all residuals taken from the previous iterate.  Rounding, which the
 * paper leaves open: A p is accumulated as diag p, then fused multiply-adds
 * of the E, W, N, S neighbours in that order; the division by the diagonal
 * is a product with its correctly rounded reciprocal 1/diag; the update is
 * one fused multiply-add.  Every check_every
 * sweeps (cycle boundaries) the convergence measure
 *   E = max_c |(rhs - A p)_c / diag_c|,
 * i.e. the size of the plain Jacobi update of eq. (32), is evaluated on the
 * current iterate; the solve stops there when E < tol (result: that iterate)
 * or when solve_max_iter sweeps are reached.  Walls are already folded into
 * the coefficients, so neighbours outside the corner range carry zero weight;
 * in a periodic direction they wrap around.
 */
/* compiled twice: with the FMA instruction where the CPU has it (fma() is
 * then one instruction), else with the library's fma(); both are exact */
__attribute__((target_clones("fma", "default")))
static int jacobi_srj(ora_t *o, const double *diag, const double *cE,
                      const double *cW, const double *cN, const double *cS,
                      const double *rhs, double *p, int32_t *sweeps,
                      double *measure) {
  const int ncx = o->ncx, ncy = o->ncy;
  const int nxc = o->nx, nyc = o->ny;
  const int px_per = per_x(o), py_per = per_y(o);
  const int nc = ncorners(o);
  double *pn = o->c[10];
  int k = 0;
  int ce = o->P.check_every > 0 ? o->P.check_every : 1;
  int kmax = o->P.solve_max_iter;
  double E = 0.0;
  int status = ORA_OK;
  /* the residual measure is relative to the right-hand side's size */
  const int resid = o->P.solve_norm == 1;
  double rmax = 0.0;
  if (resid)
    for (int c = 0; c < nc; ++c) {
      double a = fabs(rhs[c]);
      if (a > rmax) rmax = a;
    }
  for (;;) {
    int check = (k % ce == 0) || (k >= kmax);
    E = 0.0;
    double om = o->omega[k % o->n_omega];
    for (int l = 0; l < ncy; ++l)
      for (int kk = 0; kk < ncx; ++kk) {
        int c = CX(o, kk, l);
        double Ap = diag[c] * p[c];
        if (kk + 1 < ncx || px_per)
          Ap = fma(cE[c], p[CX(o, refl(kk + 1, nxc, px_per), l)], Ap);
        if (kk - 1 >= 0 || px_per)
          Ap = fma(cW[c], p[CX(o, refl(kk - 1, nxc, px_per), l)], Ap);
        if (l + 1 < ncy || py_per)
          Ap = fma(cN[c], p[CX(o, kk, refl(l + 1, nyc, py_per))], Ap);
        if (l - 1 >= 0 || py_per)
          Ap = fma(cS[c], p[CX(o, kk, refl(l - 1, nyc, py_per))], Ap);
        double upd = (rhs[c] - Ap) * (1.0 / diag[c]);  /* plain Jacobi update */
        if (check) {
          double e = resid ? fabs(rhs[c] - Ap) : fabs(upd);
          if (!(e <= E)) E = (e == e) ? e : INFINITY;
        }
        pn[c] = fma(om, upd, p[c]);
      }
    if (check && resid && rmax > 0.0) E = E / rmax;
    if (check && E < o->P.solve_tol) break;
    if (k >= kmax) {
      status = ORA_ENOCONV;
      break;
    }
    memcpy(p, pn, sizeof(double) * nc);
    ++k;
  }
  if (sweeps) *sweeps = k;
  if (measure) *measure = E;
  return status;
}

/* eq. (26)-(27) correction (1D) and eq. (36) (2D); corner w update of (28)/(41).
 * h, q ghosted and filled; outputs interior q and corner w. */
static void correct_g(ora_t *o, const double *h, const double *q1,
                      const double *q2, const double *w, const double *p,
                      double dt, double *Oq1, double *Oq2, double *Ow) {
  const int nx = o->nx, ny = o->ny;
  const double dx = o->P.dx, dy = o->P.dy, eps = o->P.dry_eps;
  double *zeta = o->b[14];
  int N = o->gx * o->gy;
  for (int n = 0; n < N; ++n) zeta[n] = h[n] - 2.0 * o->H[n];
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      int c = IX(o, i, j);
      double zx = (zeta[IX(o, i + 1, j)] - zeta[IX(o, i - 1, j)]) / (2.0 * dx);
      if (o->is1d) {
        double pR = p[i + 1], pL = p[i];
        double T = -0.5 * (h[c] * ((pR - pL) / dx) + (0.5 * (pR + pL)) * zx);
        double qn = q1[c] + dt * T;
        if (h[c] <= eps) qn = 0.0;
        Oq1[c] = qn;
        Oq2[c] = 0.0;
        continue;
      }
      double zy = (zeta[IX(o, i, j + 1)] - zeta[IX(o, i, j - 1)]) / (2.0 * dy);
      double pSW = p[CX(o, i, j)], pSE = p[CX(o, i + 1, j)];
      double pNW = p[CX(o, i, j + 1)], pNE = p[CX(o, i + 1, j + 1)];
      double TN = -0.5 * h[c] * (pNE - pNW) / dx - 0.5 * (0.5 * (pNE + pNW)) * zx;
      double TS = -0.5 * h[c] * (pSE - pSW) / dx - 0.5 * (0.5 * (pSE + pSW)) * zx;
      double TE = -0.5 * h[c] * (pNE - pSE) / dy - 0.5 * (0.5 * (pNE + pSE)) * zy;
      double TW = -0.5 * h[c] * (pNW - pSW) / dy - 0.5 * (0.5 * (pNW + pSW)) * zy;
      double a = q1[c] + dt * (0.5 * (TN + TS));
      double b = q2[c] + dt * (0.5 * (TE + TW));
      if (h[c] <= eps) {
        a = 0.0;
        b = 0.0;
      }
      Oq1[c] = a;
      Oq2[c] = b;
    }
  for (int l = 0; l < o->ncy; ++l)
    for (int k = 0; k < o->ncx; ++k) {
      double hc;
      if (o->is1d)
        hc = 0.5 * (h[IX(o, k - 1, 0)] + h[IX(o, k, 0)]);
      else
        hc = 0.25 * (h[IX(o, k - 1, l - 1)] + h[IX(o, k, l - 1)] +
                     h[IX(o, k - 1, l)] + h[IX(o, k, l)]);
      int c = CX(o, k, l);
      Ow[c] = w[c] + dt * desing_div(p[c], hc, o->P.delta);
    }
}

/* Literal constraint at every corner (for the probe assembly test). */
static double T_hor(const ora_t *o, const double *h, const double *zeta,
                    const double *p, int i, int j, int north) {
  /* T^Hor_N (north = 1) / T^Hor_S of cell (i, j), Appendix A.2 */
  int l = north ? j + 1 : j;
  double pe = P_at(o, p, i + 1, l), pw = P_at(o, p, i, l);
  double zx = (zeta[IX(o, i + 1, j)] - zeta[IX(o, i - 1, j)]) / (2.0 * o->P.dx);
  return -0.5 * h[IX(o, i, j)] * (pe - pw) / o->P.dx - 0.5 * ((pe + pw) / 2.0) * zx;
}
static double T_ver(const ora_t *o, const double *h, const double *zeta,
                    const double *p, int i, int j, int east) {
  /* T^Ver_E (east = 1) / T^Ver_W of cell (i, j), Appendix A.2 */
  int k = east ? i + 1 : i;
  double pn = P_at(o, p, k, j + 1), ps = P_at(o, p, k, j);
  double zy = (zeta[IX(o, i, j + 1)] - zeta[IX(o, i, j - 1)]) / (2.0 * o->P.dy);
  return -0.5 * h[IX(o, i, j)] * (pn - ps) / o->P.dy - 0.5 * ((pn + ps) / 2.0) * zy;
}

static void constraint_g(ora_t *o, const double *h, const double *q1,
                         const double *q2, const double *w, const double *p,
                         double dt, double *out) {
  const double dx = o->P.dx, dy = o->P.dy;
  double *zeta = o->b[14];
  int N = o->gx * o->gy;
  for (int n = 0; n < N; ++n) zeta[n] = h[n] - 2.0 * o->H[n];
  if (o->is1d) {
    /* eq. (24)-(25) at x_{k}, with cells corrected by eq. (26)-(27) */
    for (int k = 0; k <= o->nx; ++k) {
      double qc[2];
      for (int s = 0; s < 2; ++s) {
        int i = k - 1 + s;
        double pR = P_at(o, p, i + 1, 0), pL = P_at(o, p, i, 0);
        double zx =
            (zeta[IX(o, i + 1, 0)] - zeta[IX(o, i - 1, 0)]) / (2.0 * dx);
        double T = -0.5 * (h[IX(o, i, 0)] * ((pR - pL) / dx) + (0.5 * (pR + pL)) * zx);
        qc[s] = q1[IX(o, i, 0)] + dt * T;
      }
      int W = IX(o, k - 1, 0), E = IX(o, k, 0);
      double hc = 0.5 * (h[E] + h[W]);
      double qm = 0.5 * (qc[1] + qc[0]);
      double qx = (qc[1] - qc[0]) / dx;
      double zx = (zeta[E] - zeta[W]) / dx;
      /* h_c w^{n+1} = h_c w* + dt p (the h_c of w = w* + dt p / h_c cancels) */
      out[k] = hc * qx - qm * zx + 2.0 * (hc * w[k] + dt * p[k]);
    }
    return;
  }
  for (int l = 0; l <= o->ny; ++l)
    for (int k = 0; k <= o->nx; ++k) {
      /* cells: SW=(k-1,l-1) SE=(k,l-1) NW=(k-1,l) NE=(k,l) */
      double q1E = 0.5 * (q1[IX(o, k, l)] + q1[IX(o, k, l - 1)]) +
                   0.5 * dt * T_hor(o, h, zeta, p, k, l, 0) +
                   0.5 * dt * T_hor(o, h, zeta, p, k, l - 1, 1);
      double q1W = 0.5 * (q1[IX(o, k - 1, l)] + q1[IX(o, k - 1, l - 1)]) +
                   0.5 * dt * T_hor(o, h, zeta, p, k - 1, l, 0) +
                   0.5 * dt * T_hor(o, h, zeta, p, k - 1, l - 1, 1);
      double q2N = 0.5 * (q2[IX(o, k, l)] + q2[IX(o, k - 1, l)]) +
                   0.5 * dt * T_ver(o, h, zeta, p, k, l, 0) +
                   0.5 * dt * T_ver(o, h, zeta, p, k - 1, l, 1);
      double q2S = 0.5 * (q2[IX(o, k, l - 1)] + q2[IX(o, k - 1, l - 1)]) +
                   0.5 * dt * T_ver(o, h, zeta, p, k, l - 1, 0) +
                   0.5 * dt * T_ver(o, h, zeta, p, k - 1, l - 1, 1);
      double zE = 0.5 * (zeta[IX(o, k, l)] + zeta[IX(o, k, l - 1)]);
      double zW = 0.5 * (zeta[IX(o, k - 1, l)] + zeta[IX(o, k - 1, l - 1)]);
      double zN = 0.5 * (zeta[IX(o, k, l)] + zeta[IX(o, k - 1, l)]);
      double zS = 0.5 * (zeta[IX(o, k, l - 1)] + zeta[IX(o, k - 1, l - 1)]);
      double hc = 0.25 * (h[IX(o, k - 1, l - 1)] + h[IX(o, k, l - 1)] +
                          h[IX(o, k - 1, l)] + h[IX(o, k, l)]);
      double divQ = (q1E - q1W) / dx + (q2N - q2S) / dy;
      double Qx = (q1E + q1W) / 2.0, Qy = (q2N + q2S) / 2.0;
      double gzx = (zE - zW) / dx, gzy = (zN - zS) / dy;
      int c = CX(o, k, l);
      out[c] = hc * divQ - (Qx * gzx + Qy * gzy) + 2.0 * (hc * w[c] + dt * p[c]);
    }
}

/* ------------------------------------------------------------------ */
/* one projection-correction stage and the RK2 step                    */
/* ------------------------------------------------------------------ */
static int solve_g(ora_t *o, double *diag, double *cE, double *cW, double *cN,
                   double *cS, double *rhs, double *p, int32_t *sweeps,
                   double *measure) {
  if (o->is1d) {
    int st;
    if (per_x(o)) {  /* nx distinct corners; corner nx is corner 0 */
      st = thomas_cyclic(o->nx, cW, diag, cE, rhs, p, o->c[12], o->c[13],
                         o->c[10], o->c[11]);
      p[o->nx] = p[0];
    } else {
      st = thomas(o->ncx, cW, diag, cE, rhs, p, o->c[10], o->c[11]);
    }
    if (sweeps) *sweeps = 0;
    if (measure) *measure = 0.0;
    return st;
  }
  return jacobi_srj(o, diag, cE, cW, cN, cS, rhs, p, sweeps, measure);
}

static void assemble_g(ora_t *o, const double *h, const double *q1,
                       const double *q2, const double *w, double dt,
                       double *diag, double *cE, double *cW, double *cN,
                       double *cS, double *rhs) {
  if (o->is1d) {
    assemble1d_g(o, h, q1, w, dt, cW, diag, cE, rhs);
    int n = o->ncx;
    for (int k = 0; k < n; ++k) cN[k] = cS[k] = 0.0;
  } else {
    assemble2d_g(o, h, q1, q2, w, dt, diag, cE, cW, cN, cS, rhs);
  }
}

/* Manning friction (the law of Section 2: tau = g h n^2 u |u| / h^(4/3)),
 * discretised semi-implicitly as Sections 3-4 state, in this reading: on the
 * finite-volume result of each stage, in every wet cell,
 *   q <- q / (1 + dt g n^2 |u| / h^(4/3)),
 * i.e. q_t = -g n^2 |u| q / h^(4/3) with q implicit and |u|, h explicit; |u|
 * from the desingularised velocities of that result (Section 4.5). */
static void friction_g(ora_t *o, double *hs, double *q1s, double *q2s,
                       double dt) {
  const double n = o->P.manning;
  if (!(n > 0.0)) return;
  const double gn2 = o->P.g * n * n;
  for (int j = 0; j < (o->is1d ? 1 : o->ny); ++j)
    for (int i = 0; i < o->nx; ++i) {
      const int c = IX(o, i, j);
      const double h = hs[c];
      if (h <= o->P.dry_eps) continue;
      const double u = ora_desing_velocity(h, q1s[c], o->P.delta);
      const double v =
          o->is1d ? 0.0 : ora_desing_velocity(h, q2s[c], o->P.delta);
      const double den = 1.0 + dt * gn2 * sqrt(u * u + v * v) / (h * cbrt(h));
      q1s[c] = q1s[c] / den;
      if (!o->is1d) q2s[c] = q2s[c] / den;
    }
}

/* Energy-consistent vertical momentum (the form named after eq. 7):
 * (hw)_t + div(hw u) = p.  With the mass equation h_t + div(h u) = 0 this is
 * h (w_t + u . grad w) = p, so the variant adds the transport of w by the
 * flow to the hyperbolic step of each stage; the projection step is the
 * model's, w = w* + dt p / h_c.  Reading (the paper gives no discretisation
 * for it): w lives at the corners; the corner velocity is the desingularised
 * (Section 4.5) ratio of the means of q and h over the cells around the
 * corner (of the stage input V, ghosted); the transport is first-order
 * upwind in each direction,
 *   w* = w - dt [ u+ (w_k - w_{k-1})/dx + u- (w_{k+1} - w_k)/dx
 *                + v+ (w_l - w_{l-1})/dy + v- (w_{l+1} - w_l)/dy ],
 * u+ = max(u, 0), u- = min(u, 0); corners beyond a wall or an open side are
 * reflected as the pressure's are, wrapped on a periodic line; a dry corner
 * (h_c <= dry_eps) keeps its w.  It keeps a uniform w uniform, and for a
 * uniform current on a periodic line it moves the first moment of w by
 * exactly u dt per step. */
static void advect_w_g(const ora_t *o, const double *Vh, const double *Vq1,
                       const double *Vq2, const double *w_in, double dt,
                       double *w_out) {
  const double dx = o->P.dx, dy = o->P.dy, de = o->P.delta;
  for (int l = 0; l < o->ncy; ++l)
    for (int k = 0; k < o->ncx; ++k) {
      double hc, qc1, qc2 = 0.0;
      if (o->is1d) {
        hc = 0.5 * (Vh[IX(o, k - 1, 0)] + Vh[IX(o, k, 0)]);
        qc1 = 0.5 * (Vq1[IX(o, k - 1, 0)] + Vq1[IX(o, k, 0)]);
      } else {
        hc = 0.25 * (Vh[IX(o, k - 1, l - 1)] + Vh[IX(o, k, l - 1)] +
                     Vh[IX(o, k - 1, l)] + Vh[IX(o, k, l)]);
        qc1 = 0.25 * (Vq1[IX(o, k - 1, l - 1)] + Vq1[IX(o, k, l - 1)] +
                      Vq1[IX(o, k - 1, l)] + Vq1[IX(o, k, l)]);
        qc2 = 0.25 * (Vq2[IX(o, k - 1, l - 1)] + Vq2[IX(o, k, l - 1)] +
                      Vq2[IX(o, k - 1, l)] + Vq2[IX(o, k, l)]);
      }
      const int c = CX(o, k, l);
      const double w = w_in[c];
      if (hc <= o->P.dry_eps) {
        w_out[c] = w;
        continue;
      }
      const double u = ora_desing_velocity(hc, qc1, de);
      const double ddx =
          u > 0.0 ? (w - P_at(o, w_in, k - 1, l)) / dx
                  : (P_at(o, w_in, k + 1, l) - w) / dx;
      double adv = u * ddx;
      if (!o->is1d) {
        const double v = ora_desing_velocity(hc, qc2, de);
        const double ddy =
            v > 0.0 ? (w - P_at(o, w_in, k, l - 1)) / dy
                    : (P_at(o, w_in, k, l + 1) - w) / dy;
        adv = adv + v * ddy;
      }
      w_out[c] = w - dt * adv;
    }
}

/* Stage: V (ghosted, filled) + corner w_in, warm start p -> outputs. */
static int stage_g(ora_t *o, const double *Vh, const double *Vq1,
                   const double *Vq2, const double *w_in, double *p, double dt,
                   double *Oh, double *Oq1, double *Oq2, double *Ow,
                   int32_t *sweeps, double *measure) {
  double *hs = o->b[0], *q1s = o->b[1], *q2s = o->b[2];
  int N = o->gx * o->gy, nc = ncorners(o);
  memset(hs, 0, sizeof(double) * N);
  memset(q1s, 0, sizeof(double) * N);
  memset(q2s, 0, sizeof(double) * N);
  fv_stage_g(o, Vh, Vq1, Vq2, dt, hs, q1s, q2s, &o->clamped_total);
  friction_g(o, hs, q1s, q2s, dt);
  fill_ghosts(o, hs, 1.0, 1.0);
  fill_ghosts(o, q1s, -1.0, 1.0);
  fill_ghosts(o, q2s, 1.0, -1.0);
  double *ws = o->c[0];
  if (o->P.w_advection)
    advect_w_g(o, Vh, Vq1, Vq2, w_in, dt, ws);
  else
    memcpy(ws, w_in, sizeof(double) * nc);
  if (o->P.breaking_on) breaking_g(o, hs, q1s, q2s, ws, dt);
  int st = ORA_OK;
  *sweeps = 0;
  *measure = 0.0;
  if (o->P.nh_on) {
    double *diag = o->c[1], *cE = o->c[2], *cW = o->c[3], *cN = o->c[4],
           *cS = o->c[5], *rhs = o->c[6];
    assemble_g(o, hs, q1s, q2s, ws, dt, diag, cE, cW, cN, cS, rhs);
    /* Gershgorin check of Section 5, reported (not enforced): the dominance
     * margin 16 + ... depends on the curvature of zeta and can be lost. */
    for (int c = 0; c < nc; ++c) {
      double off = fabs(cE[c]) + fabs(cW[c]) + fabs(cN[c]) + fabs(cS[c]);
      if (!(diag[c] > off)) o->nondom_last += 1;
    }
    int s2 = solve_g(o, diag, cE, cW, cN, cS, rhs, p, sweeps, measure);
    if (s2 != ORA_OK && st == ORA_OK) st = s2;
    correct_g(o, hs, q1s, q2s, ws, p, dt, Oq1, Oq2, Ow);
    for (int n = 0; n < N; ++n) Oh[n] = hs[n];
  } else {
    for (int n = 0; n < N; ++n) {
      Oh[n] = hs[n];
      Oq1[n] = q1s[n];
      Oq2[n] = q2s[n];
    }
    memcpy(Ow, ws, sizeof(double) * nc);
  }
  fill_ghosts(o, Oh, 1.0, 1.0);
  fill_ghosts(o, Oq1, -1.0, 1.0);
  fill_ghosts(o, Oq2, 1.0, -1.0);
  return st;
}

/*
 * One time step: second-order TVD Runge-Kutta (Heun form) in which each stage
 * is the full projection-correction step (FV, breaking, pressure, correction):
 *   U1 = Pi(U^n + dt L(U^n)),  U2 = Pi(U1 + dt L(U1)),
 *   U^{n+1} = (U^n + U2)/2,    w^{n+1} = (w^n + w2)/2,  p^{n+1} = p2
 * (reading of Section 6, which repeats its steps 1-4 twice).  The next dt comes
 * from the CFL condition on U^{n+1}.
 */
/* Generation/absorption zones of Section 4.4, on every wall with a width
 * L > 0, in this reading: the zone holds the k + 1 cells nearest the wall,
 * k the least natural number with k dx >= L; a cell at distance d from the
 * zone's innermost cell (d = 0 .. k dx) gets m = sqrt(max(0, 1 - (d/L)^2)),
 * so m = 1 at the inner edge and 0 at the wall cell (the paper states this
 * for the right end; the left end mirrors it).  Cells outside every zone have
 * m = 1; in 2D the weights of x and y multiply (each side relaxed in turn).
 * A corner takes the mean of the two cells beside it per direction (mirrored
 * at walls).  After each step: U <- m U + (1 - m) U*, w and p likewise with
 * the corner weights. */
/* the cell whose mirror image sits at index i (walls) */
static int cell_mirror(int i, int n) {
  return i < 0 ? -1 - i : (i >= n ? 2 * n - 1 - i : i);
}

static void zone_weights(int n, double dx, double Llo, double Lhi, double *m) {
  for (int i = 0; i < n; ++i) m[i] = 1.0;
  const double L[2] = {Llo, Lhi};
  for (int side = 0; side < 2; ++side) {
    if (!(L[side] > 0.0)) continue;
    int k = (int)ceil(L[side] / dx);
    while (k > 0 && (k - 1) * dx >= L[side]) --k;  /* least k: k dx >= L */
    for (int r = 0; r <= k && r < n; ++r) {        /* r: cells from inner */
      const int i = side == 0 ? k - r : n - 1 - k + r;
      if (i < 0 || i >= n) continue;
      const double d = r * dx / L[side];
      m[i] *= sqrt(dmax(0.0, 1.0 - d * d));
    }
  }
}

int ora_set_relaxation(ora_t *o, const double *widths, const double *h_t,
                       const double *q1_t, const double *q2_t,
                       const double *w_t, const double *p_t) {
  if (!o || !widths) return ORA_EINVAL;
  for (int s = 0; s < 4; ++s)
    if (!(widths[s] >= 0.0) || isinf(widths[s])) return ORA_EINVAL;
  /* zones lie along walls: none across a periodic direction */
  if (per_x(o) && (widths[0] > 0.0 || widths[1] > 0.0)) return ORA_EINVAL;
  if (per_y(o) && (widths[2] > 0.0 || widths[3] > 0.0)) return ORA_EINVAL;
  const int N = o->gx * o->gy, nc = ncorners(o);
  double **arrs[7] = {&o->rm_cell, &o->rm_corn, &o->rt_h, &o->rt_q1,
                      &o->rt_q2,   &o->rt_w,    &o->rt_p};
  for (int a = 0; a < 7; ++a) {
    free(*arrs[a]);
    *arrs[a] = NULL;
  }
  if (!(widths[0] > 0 || widths[1] > 0 ||
        (!o->is1d && (widths[2] > 0 || widths[3] > 0))))
    return ORA_OK;  /* no zone: off */
  double *mx = (double *)malloc(sizeof(double) * o->nx);
  double *my = (double *)malloc(sizeof(double) * (o->is1d ? 1 : o->ny));
  zone_weights(o->nx, o->P.dx, widths[0], widths[1], mx);
  if (o->is1d)
    my[0] = 1.0;
  else
    zone_weights(o->ny, o->P.dy, widths[2], widths[3], my);
  o->rm_cell = (double *)calloc(N, sizeof(double));
  o->rm_corn = (double *)calloc(nc, sizeof(double));
  o->rt_h = (double *)calloc(N, sizeof(double));
  o->rt_q1 = (double *)calloc(N, sizeof(double));
  o->rt_q2 = (double *)calloc(N, sizeof(double));
  o->rt_w = (double *)calloc(nc, sizeof(double));
  o->rt_p = (double *)calloc(nc, sizeof(double));
  const int ny = o->is1d ? 1 : o->ny;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < o->nx; ++i) {
      const int c = IX(o, i, j), f = j * o->nx + i;
      o->rm_cell[c] = mx[i] * my[j];
      /* still water by default: eta* = 0 (h* = H, none on land), q* = 0 */
      o->rt_h[c] = h_t ? h_t[f] : dmax(o->H[c], 0.0);
      o->rt_q1[c] = q1_t ? q1_t[f] : 0.0;
      o->rt_q2[c] = q2_t ? q2_t[f] : 0.0;
    }
  for (int l = 0; l < o->ncy; ++l)
    for (int k = 0; k < o->ncx; ++k) {
      const int c = CX(o, k, l);
      const double ax =
          0.5 * (mx[cell_mirror(k - 1, o->nx)] + mx[cell_mirror(k, o->nx)]);
      const double ay = o->is1d ? 1.0
                                : 0.5 * (my[cell_mirror(l - 1, o->ny)] +
                                         my[cell_mirror(l, o->ny)]);
      o->rm_corn[c] = ax * ay;
      o->rt_w[c] = w_t ? w_t[c] : 0.0;
      o->rt_p[c] = p_t ? p_t[c] : 0.0;
    }
  free(mx);
  free(my);
  return ORA_OK;
}

static void relax_g(ora_t *o) {
  if (!o->rm_cell) return;
  const int ny = o->is1d ? 1 : o->ny;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < o->nx; ++i) {
      const int c = IX(o, i, j);
      const double m = o->rm_cell[c];
      o->h[c] = m * o->h[c] + (1.0 - m) * o->rt_h[c];
      o->q1[c] = m * o->q1[c] + (1.0 - m) * o->rt_q1[c];
      o->q2[c] = m * o->q2[c] + (1.0 - m) * o->rt_q2[c];
    }
  for (int c = 0; c < ncorners(o); ++c) {
    const double m = o->rm_corn[c];
    o->w[c] = m * o->w[c] + (1.0 - m) * o->rt_w[c];
    o->p[c] = m * o->p[c] + (1.0 - m) * o->rt_p[c];
  }
  /* the wall ghosts image the relaxed state */
  fill_ghosts(o, o->h, 1.0, 1.0);
  fill_ghosts(o, o->q1, -1.0, 1.0);
  fill_ghosts(o, o->q2, 1.0, -1.0);
}

int ora_step(ora_t *o) {
  int N = o->gx * o->gy, nc = ncorners(o);
  double dt = o->P.fixed_dt ? o->P.dt_fixed : o->dt;
  if (!(dt > 0.0) || !isfinite(dt)) {
    o->last_status = ORA_EINVAL;
    return ORA_EINVAL;
  }
  double *h1 = o->b[3], *q11 = o->b[4], *q21 = o->b[5];
  double *h2 = o->b[6], *q12 = o->b[7], *q22 = o->b[15];
  double *w1 = o->c[7], *w2 = o->c[8];
  int32_t s1 = 0, s2 = 0;
  double m1 = 0.0, m2 = 0.0;
  o->nondom_last = 0;
  int st = stage_g(o, o->h, o->q1, o->q2, o->w, o->p, dt, h1, q11, q21, w1, &s1,
                   &m1);
  int stb = stage_g(o, h1, q11, q21, w1, o->p, dt, h2, q12, q22, w2, &s2, &m2);
  if (st == ORA_OK) st = stb;
  for (int n = 0; n < N; ++n) {
    o->h[n] = 0.5 * (o->h[n] + h2[n]);
    o->q1[n] = 0.5 * (o->q1[n] + q12[n]);
    o->q2[n] = 0.5 * (o->q2[n] + q22[n]);
  }
  for (int c = 0; c < nc; ++c) o->w[c] = 0.5 * (o->w[c] + w2[c]);
  relax_g(o);
  o->t += dt;
  o->dt_last = dt;
  o->step += 1;
  o->sweeps_stage[0] = s1;
  o->sweeps_stage[1] = s2;
  o->sweeps_total += s1 + s2;
  o->solves_total += o->P.nh_on ? 2 : 0;
  o->measure_last = m2;
  for (int j = 0; j < o->ny; ++j)
    for (int i = 0; i < o->nx; ++i) {
      int c = IX(o, i, j);
      if (!isfinite(o->h[c]) || !isfinite(o->q1[c]) || !isfinite(o->q2[c]))
        st = ORA_ENONFINITE;
    }
  if (!o->P.fixed_dt) o->dt = cfl_dt_g(o, o->h, o->q1, o->q2);
  o->last_status = st;
  return st;
}

int ora_run(ora_t *o, int64_t nsteps) {
  for (int64_t n = 0; n < nsteps; ++n) {
    int st = ora_step(o);
    if (st != ORA_OK) return st;
  }
  return ORA_OK;
}

/* ------------------------------------------------------------------ */
/* lifecycle                                                           */
/* ------------------------------------------------------------------ */
ora_t *ora_create(const ora_params *pp, const double *omega, int32_t n_omega) {
  /* mirror ghosts need at least two interior cells per direction */
  if (!pp || pp->nx < 2 || pp->ny < 1 || !(pp->dx > 0) || !(pp->dy > 0))
    return NULL;
  if (!(pp->manning >= 0.0) || isinf(pp->manning)) return NULL;
  if (pp->open_sides < 0 || pp->open_sides > 15) return NULL;
  if (pp->periodic < 0 || pp->periodic > 3) return NULL;
  if (pp->w_advection < 0 || pp->w_advection > 1) return NULL;
  if (pp->solve_norm < 0 || pp->solve_norm > 1) return NULL;
  /* a periodic direction has no ends: no open side in it */
  if ((pp->periodic & 1) && (pp->open_sides & 3)) return NULL;
  if (pp->ny > 1 && (pp->periodic & 2) && (pp->open_sides & 12)) return NULL;
  ora_t *o = (ora_t *)calloc(1, sizeof(ora_t));
  o->P = *pp;
  o->is1d = pp->ny == 1;
  o->nx = pp->nx;
  o->ny = pp->ny;
  o->gx = pp->nx + 2 * GH;
  o->gy = o->is1d ? 1 : pp->ny + 2 * GH;
  o->goy = o->is1d ? 0 : GH;
  o->ncx = pp->nx + 1;
  o->ncy = o->is1d ? 1 : pp->ny + 1;
  if (n_omega <= 0 || !omega) {
    o->n_omega = 1;
    o->omega = (double *)malloc(sizeof(double));
    o->omega[0] = 1.0;
  } else {
    o->n_omega = n_omega;
    o->omega = (double *)malloc(sizeof(double) * n_omega);
    memcpy(o->omega, omega, sizeof(double) * n_omega);
  }
  size_t N = (size_t)o->gx * o->gy, nc = (size_t)o->ncx * o->ncy;
  o->H = (double *)calloc(N, sizeof(double));
  o->h = (double *)calloc(N, sizeof(double));
  o->q1 = (double *)calloc(N, sizeof(double));
  o->q2 = (double *)calloc(N, sizeof(double));
  o->w = (double *)calloc(nc, sizeof(double));
  o->p = (double *)calloc(nc, sizeof(double));
  for (int m = 0; m < 16; ++m) {
    o->b[m] = (double *)calloc(N, sizeof(double));
    o->c[m] = (double *)calloc(nc, sizeof(double));
  }
  return o;
}

void ora_destroy(ora_t *o) {
  if (!o) return;
  free(o->omega);
  free(o->H);
  free(o->h);
  free(o->q1);
  free(o->q2);
  free(o->w);
  free(o->p);
  for (int m = 0; m < 16; ++m) {
    free(o->b[m]);
    free(o->c[m]);
  }
  free(o->rm_cell);
  free(o->rm_corn);
  free(o->rt_h);
  free(o->rt_q1);
  free(o->rt_q2);
  free(o->rt_w);
  free(o->rt_p);
  free(o);
}

int ora_set_bathymetry(ora_t *o, const double *H) {
  load_cells(o, o->H, H);
  fill_ghosts(o, o->H, 1.0, 1.0);
  return ORA_OK;
}

int ora_set_state(ora_t *o, const double *h, const double *q1,
                  const double *q2, const double *w, const double *p) {
  int nc = ncorners(o);
  load_cells(o, o->h, h);
  for (int j = 0; j < o->ny; ++j)
    for (int i = 0; i < o->nx; ++i)
      if (o->h[IX(o, i, j)] < 0.0) return ORA_ENEGDEPTH;
  load_cells(o, o->q1, q1);
  if (q2 && !o->is1d)
    load_cells(o, o->q2, q2);
  else
    memset(o->q2, 0, sizeof(double) * o->gx * o->gy);
  fill_ghosts(o, o->h, 1.0, 1.0);
  fill_ghosts(o, o->q1, -1.0, 1.0);
  fill_ghosts(o, o->q2, 1.0, -1.0);
  if (w)
    memcpy(o->w, w, sizeof(double) * nc);
  else
    memset(o->w, 0, sizeof(double) * nc);
  if (p)
    memcpy(o->p, p, sizeof(double) * nc);
  else
    memset(o->p, 0, sizeof(double) * nc);
  o->t = 0.0;
  o->step = 0;
  o->clamped_total = 0.0;
  o->sweeps_total = 0;
  o->solves_total = 0;
  o->dt = o->P.fixed_dt ? o->P.dt_fixed : cfl_dt_g(o, o->h, o->q1, o->q2);
  return ORA_OK;
}

int ora_get_state(const ora_t *o, double *h, double *q1, double *q2,
                  double *w, double *p) {
  int nc = ncorners(o);
  if (h) store_cells(o, h, o->h);
  if (q1) store_cells(o, q1, o->q1);
  if (q2) store_cells(o, q2, o->q2);
  if (w) memcpy(w, o->w, sizeof(double) * nc);
  if (p) memcpy(p, o->p, sizeof(double) * nc);
  return ORA_OK;
}

void ora_get_stats(const ora_t *o, double *s) {
  s[0] = o->t;
  s[1] = o->P.fixed_dt ? o->P.dt_fixed : o->dt;
  s[2] = (double)o->step;
  s[3] = (double)o->sweeps_stage[0];
  s[4] = (double)o->sweeps_stage[1];
  s[5] = o->measure_last;
  s[6] = o->clamped_total;
  s[7] = (double)o->sweeps_total;
  s[8] = (double)o->solves_total;
  s[9] = o->dt_last;
  s[10] = (double)o->last_status;
  s[11] = (double)o->nondom_last;
}

/* ---- component wrappers: load into ghosted buffers, compute, store ---- */
static void load_state_g(ora_t *o, const double *h, const double *q1,
                         const double *q2, double *gh, double *gq1,
                         double *gq2) {
  int N = o->gx * o->gy;
  memset(gh, 0, sizeof(double) * N);
  memset(gq1, 0, sizeof(double) * N);
  memset(gq2, 0, sizeof(double) * N);
  load_cells(o, gh, h);
  load_cells(o, gq1, q1);
  if (q2 && !o->is1d) load_cells(o, gq2, q2);
  fill_ghosts(o, gh, 1.0, 1.0);
  fill_ghosts(o, gq1, -1.0, 1.0);
  fill_ghosts(o, gq2, 1.0, -1.0);
}

double ora_cfl_dt(ora_t *o, const double *h, const double *q1,
                  const double *q2) {
  load_state_g(o, h, q1, q2, o->b[3], o->b[4], o->b[5]);
  return cfl_dt_g(o, o->b[3], o->b[4], o->b[5]);
}

int ora_fv_stage(ora_t *o, const double *h, const double *q1, const double *q2,
                 double dt, double *h_out, double *q1_out, double *q2_out,
                 double *clamped) {
  load_state_g(o, h, q1, q2, o->b[3], o->b[4], o->b[5]);
  double cl = 0.0;
  fv_stage_g(o, o->b[3], o->b[4], o->b[5], dt, o->b[6], o->b[7], o->b[15], &cl);
  store_cells(o, h_out, o->b[6]);
  store_cells(o, q1_out, o->b[7]);
  if (q2_out) store_cells(o, q2_out, o->b[15]);
  if (clamped) *clamped = cl;
  return ORA_OK;
}

int ora_breaking(ora_t *o, const double *h, double *q1, double *q2, double *w,
                 double dt) {
  load_state_g(o, h, q1, q2, o->b[3], o->b[4], o->b[5]);
  breaking_g(o, o->b[3], o->b[4], o->b[5], w, dt);
  store_cells(o, q1, o->b[4]);
  if (q2 && !o->is1d) store_cells(o, q2, o->b[5]);
  return ORA_OK;
}

int ora_assemble(ora_t *o, const double *h, const double *q1, const double *q2,
                 const double *w, double dt, double *diag, double *cE,
                 double *cW, double *cN, double *cS, double *rhs) {
  load_state_g(o, h, q1, q2, o->b[3], o->b[4], o->b[5]);
  assemble_g(o, o->b[3], o->b[4], o->b[5], w, dt, diag, cE, cW, cN, cS, rhs);
  return ORA_OK;
}

int ora_constraint(ora_t *o, const double *h, const double *q1,
                   const double *q2, const double *w, const double *p,
                   double dt, double *out) {
  load_state_g(o, h, q1, q2, o->b[3], o->b[4], o->b[5]);
  constraint_g(o, o->b[3], o->b[4], o->b[5], w, p, dt, out);
  return ORA_OK;
}

int ora_solve(ora_t *o, const double *diag, const double *cE, const double *cW,
              const double *cN, const double *cS, const double *rhs, double *p,
              int32_t *sweeps, double *measure) {
  return solve_g(o, (double *)diag, (double *)cE, (double *)cW, (double *)cN,
                 (double *)cS, (double *)rhs, p, sweeps, measure);
}

int ora_dense_solve(ora_t *o, const double *diag, const double *cE,
                    const double *cW, const double *cN, const double *cS,
                    const double *rhs, double *p) {
  int n = ncorners(o);
  if (n > 4096) return ORA_EINVAL;
  double *A = (double *)calloc((size_t)n * n, sizeof(double));
  double *b = (double *)malloc(sizeof(double) * n);
  for (int l = 0; l < o->ncy; ++l)
    for (int k = 0; k < o->ncx; ++k) {
      int c = CX(o, k, l);
      const int px_per = per_x(o), py_per = per_y(o);
      A[(size_t)c * n + c] = diag[c];
      if (k + 1 < o->ncx || px_per)
        A[(size_t)c * n + CX(o, refl(k + 1, o->nx, px_per), l)] += cE[c];
      if (k - 1 >= 0 || px_per)
        A[(size_t)c * n + CX(o, refl(k - 1, o->nx, px_per), l)] += cW[c];
      if (!o->is1d && (l + 1 < o->ncy || py_per))
        A[(size_t)c * n + CX(o, k, refl(l + 1, o->ny, py_per))] += cN[c];
      if (!o->is1d && (l - 1 >= 0 || py_per))
        A[(size_t)c * n + CX(o, k, refl(l - 1, o->ny, py_per))] += cS[c];
      b[c] = rhs[c];
    }
  int st = ORA_OK;
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (fabs(A[(size_t)r * n + col]) > fabs(A[(size_t)piv * n + col])) piv = r;
    if (A[(size_t)piv * n + col] == 0.0) {
      st = ORA_ENODOM;
      break;
    }
    if (piv != col) {
      for (int m = 0; m < n; ++m) {
        double t = A[(size_t)col * n + m];
        A[(size_t)col * n + m] = A[(size_t)piv * n + m];
        A[(size_t)piv * n + m] = t;
      }
      double t = b[col];
      b[col] = b[piv];
      b[piv] = t;
    }
    for (int r = col + 1; r < n; ++r) {
      double f = A[(size_t)r * n + col] / A[(size_t)col * n + col];
      if (f == 0.0) continue;
      for (int m = col; m < n; ++m) A[(size_t)r * n + m] -= f * A[(size_t)col * n + m];
      b[r] -= f * b[col];
    }
  }
  if (st == ORA_OK)
    for (int r = n - 1; r >= 0; --r) {
      double s = b[r];
      for (int m = r + 1; m < n; ++m) s -= A[(size_t)r * n + m] * p[m];
      p[r] = s / A[(size_t)r * n + r];
    }
  free(A);
  free(b);
  return st;
}

int ora_correct(ora_t *o, const double *h, const double *q1, const double *q2,
                const double *w, const double *p, double dt, double *q1_out,
                double *q2_out, double *w_out) {
  load_state_g(o, h, q1, q2, o->b[3], o->b[4], o->b[5]);
  correct_g(o, o->b[3], o->b[4], o->b[5], w, p, dt, o->b[6], o->b[7], w_out);
  store_cells(o, q1_out, o->b[6]);
  if (q2_out) store_cells(o, q2_out, o->b[7]);
  return ORA_OK;
}
