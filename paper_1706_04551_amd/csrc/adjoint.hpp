// adjoint.hpp -- device code of the adjoint (reverse) time step.
//
// The adjoint of one projection-correction stage is assembled from local
// transposed Jacobian products, each written out in reverse mode from the
// forward formulas of kernels.hpp: the flux (prim, reconstruct, pvm,
// interior), the pressure rows (assemble_row) and the correction
// (correct_cell, correct_corner).  The forward values are recomputed with
// those very functions where a branch depends on them, so every branch
// (limiter, HLL speeds, wet/dry tests, clamps) takes the forward's decision.
// The products are gathered: one thread per input cell or corner visits
// every output that reads it, so no two threads add into the same place and
// the result does not depend on scheduling.
//
// Pressure: the stage solves A(U) p = rhs(U).  With A^T mu = pbar (pbar the
// adjoint of p), the adjoint of U gains mu^T d(rhs - A p)/dU at fixed p.
#pragma once
#include "kernels.hpp"

namespace nh {

// Sums over outputs are FP64.  The flux cotangents are formed in the bulk
// type (their arithmetic dominates), those of the rows and the correction
// in FP64.
using E = double;

struct AdjGeom {
  int nx, ny;
  double dx, dy, g, delta, dry_eps;
  const double* dtp;
};

// ---------------------------------------------------------------------------
// finite-volume stage: (h*, q*) = FV(h, q; H), one direction per pass
// (DIR = 1: x, 2: y).  Along the direction a cell's flux sum is
//   f_i = Dm(i | i+1) + Dp(i-1 | i) + I_i,   out_i = U_i - dt f_i / dx + ...,
// with the edge fluctuations (eq. 18-19) of the reconstructed states of the
// two cells beside the edge (eq. 21) and the volume term I_i (eq. 22, 30).
// Reverse mode, gathered: the thread of input cell j slides along j's line
// over the edges and volume terms whose reconstructions read j, and carries
// the adjoint weights of their output cells back through them (the forward
// values, hence every branch, are those of the forward formulas):
//   edge and volume term -> cotangents of the two faces of each cell,
//   faces -> primitive values (h, un, ut, eta) of the 3 cells of the
//   reconstruction, primitives -> (h, q1, q2, H) of j.
// Next to a wall the mirrored ghost positions of j are carried too (their
// normal discharge is -q of j).  The x pass adds j's own identity term;
// hs_out (the stored h*) gives the forward's clamp and dry decisions.
// Derivative conventions: sqrt' = 0 at 0, |x|' = 1 at 0.
// ---------------------------------------------------------------------------
template <typename V>
struct FaceBar {
  V h, qn, qt, un, ut, eta;
};

template <typename V>
__device__ __forceinline__ void zero(FaceBar<V>& b) {
  b.h = b.qn = b.qt = b.un = b.ut = b.eta = V(0);
}

// cotangent of the primitive values of one cell
template <typename V>
struct PrimBar {
  V h, un, ut, eta;
};

template <typename V>
__device__ __forceinline__ V dsqrt(V r) {  // d sqrt(x)/dx at sqrt(x) = r
  return r > V(0) ? V(0.5) / r : V(0);
}

template <typename V>
__device__ __forceinline__ V dabs(V x) {
  return x < V(0) ? V(-1) : V(1);
}

// adds wL . d Dm + wR . d Dp (eq. 18-19, the forward pvm) to the faces'
// cotangents
template <typename T>
__device__ __forceinline__ void pvm_rev(const Face<T>& L, const Face<T>& R,
                                        T g, T dry_eps, const T wL[3],
                                        const T wR[3], FaceBar<T>& bL,
                                        FaceBar<T>& bR) {
  if (L.h <= dry_eps && R.h <= dry_eps) return;
  const T he = T(0.5) * (L.h + R.h);
  const T sL = sqrt(L.h), sR = sqrt(R.h);
  const T den = sL + sR;
  const T ue = (L.un * sL + R.un * sR) / den;
  const T ce = sqrt(g * he);
  const T cL = sqrt(g * L.h), cR = sqrt(g * R.h);
  const T SLa = ue - ce, SLb = L.un - cL;
  const T SRa = ue + ce, SRb = R.un + cR;
  const bool slA = SLa < SLb, srA = SRa > SRb;  // tmin, tmax picks
  const T SL = slA ? SLa : SLb, SR = srA ? SRa : SRb;
  if (!(SR - SL > T(0))) return;
  const T D = SR - SL;
  const T aSL = fabs(SL), aSR = fabs(SR);
  const T a0 = (SR * aSL - SL * aSR) / D;
  const T a1 = (aSR - aSL) / D;
  T deta = R.eta - L.eta;
  bool eta_on = true;
  if (R.h <= dry_eps && L.eta < -R.H) eta_on = false;
  if (L.h <= dry_eps && R.eta < -L.H) eta_on = false;
  if (!eta_on) deta = T(0);
  T Rv[3], dU[3];
  Rv[0] = R.qn - L.qn;
  Rv[1] = (R.qn * R.un - L.qn * L.un) + g * he * deta;
  Rv[2] = R.qn * R.ut - L.qn * L.ut;
  dU[0] = deta;
  dU[1] = R.qn - L.qn;
  dU[2] = R.qt - L.qt;
  // S = sum_m Dm_m wL_m + Dp_m wR_m
  //   = 1/2 sum_m Rv_m (wL + wR)_m + a1 Rv_m (wR - wL)_m + a0 dU_m (wR - wL)_m
  T Rvb[3], dUb[3], a0b = T(0), a1b = T(0);
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    const T sw = wL[m] + wR[m], dw = wR[m] - wL[m];
    Rvb[m] = T(0.5) * (sw + a1 * dw);
    dUb[m] = T(0.5) * a0 * dw;
    a1b = a1b + T(0.5) * Rv[m] * dw;
    a0b = a0b + T(0.5) * dU[m] * dw;
  }
  T heb = Rvb[1] * g * deta, detab = Rvb[1] * g * he + dUb[0];
  bR.qn = bR.qn + Rvb[0] + Rvb[1] * R.un + Rvb[2] * R.ut + dUb[1];
  bL.qn = bL.qn - Rvb[0] - Rvb[1] * L.un - Rvb[2] * L.ut - dUb[1];
  bR.un = bR.un + Rvb[1] * R.qn;
  bL.un = bL.un - Rvb[1] * L.qn;
  bR.ut = bR.ut + Rvb[2] * R.qn;
  bL.ut = bL.ut - Rvb[2] * L.qn;
  bR.qt = bR.qt + dUb[2];
  bL.qt = bL.qt - dUb[2];
  if (eta_on) {
    bR.eta = bR.eta + detab;
    bL.eta = bL.eta - detab;
  }
  // a0, a1 of the speeds
  const T gL = dabs(SL), gR = dabs(SR);
  const T SRbar = (a0b * (aSL - SL * gR - a0) + a1b * (gR - a1)) / D;
  const T SLbar = (a0b * (SR * gL - aSR + a0) + a1b * (a1 - gL)) / D;
  T ueb = T(0), ceb = T(0);
  if (slA) {
    ueb = ueb + SLbar;
    ceb = ceb - SLbar;
  } else {
    bL.un = bL.un + SLbar;
    bL.h = bL.h - SLbar * g * dsqrt(cL);
  }
  if (srA) {
    ueb = ueb + SRbar;
    ceb = ceb + SRbar;
  } else {
    bR.un = bR.un + SRbar;
    bR.h = bR.h + SRbar * g * dsqrt(cR);
  }
  heb = heb + ceb * g * dsqrt(ce);
  bL.un = bL.un + ueb * sL / den;
  bR.un = bR.un + ueb * sR / den;
  bL.h = bL.h + ueb * (L.un - ue) / den * dsqrt(sL) + T(0.5) * heb;
  bR.h = bR.h + ueb * (R.un - ue) / den * dsqrt(sR) + T(0.5) * heb;
}

// adds w . d I (the forward interior) to the faces' cotangents and to h0's
template <typename T>
__device__ __forceinline__ void interior_rev(const Face<T>& L,
                                             const Face<T>& R, T h0, T g,
                                             const T w[3], FaceBar<T>& bL,
                                             FaceBar<T>& bR, T& h0b) {
  bR.qn = bR.qn + w[0] + w[1] * R.un + w[2] * R.ut;
  bL.qn = bL.qn - w[0] - w[1] * L.un - w[2] * L.ut;
  bR.un = bR.un + w[1] * R.qn;
  bL.un = bL.un - w[1] * L.qn;
  bR.ut = bR.ut + w[2] * R.qn;
  bL.ut = bL.ut - w[2] * L.qn;
  h0b = h0b + w[1] * g * (R.eta - L.eta);
  bR.eta = bR.eta + w[1] * g * h0;
  bL.eta = bL.eta - w[1] * g * h0;
}

// which argument the forward minmod returned: 1 = a, 2 = b, 0 = neither
template <typename T>
__device__ __forceinline__ int minmod_pick(T a, T b) {
  if (a > T(0) && b > T(0)) return a < b ? 1 : 2;
  if (a < T(0) && b < T(0)) return a > b ? 1 : 2;
  return 0;
}

// reverse of reconstruct(m, c, p): face cotangents -> the cotangents of the
// primitive values of m, c, p (added)
template <typename T>
__device__ __forceinline__ void reconstruct_rev(
    const Prim<T>& m, const Prim<T>& c, const Prim<T>& p, T dry_eps,
    const Face<T>& L, const Face<T>& R, FaceBar<T> bL, FaceBar<T> bR,
    PrimBar<T>& bm, PrimBar<T>& bc, PrimBar<T>& bp) {
  // qn = h un, qt = h ut on each face
  bR.h = bR.h + bR.qn * R.un + bR.qt * R.ut;
  bR.un = bR.un + bR.qn * R.h;
  bR.ut = bR.ut + bR.qt * R.h;
  bL.h = bL.h + bL.qn * L.un + bL.qt * L.ut;
  bL.un = bL.un + bL.qn * L.h;
  bL.ut = bL.ut + bL.qt * L.h;
  // R = c + s/2, L = c - s/2 for each of h, eta, un, ut
  bc.h = bc.h + bR.h + bL.h;
  bc.eta = bc.eta + bR.eta + bL.eta;
  bc.un = bc.un + bR.un + bL.un;
  bc.ut = bc.ut + bR.ut + bL.ut;
  // slope = p - c (pick 1) or c - m (pick 2) or 0
  auto slope = [&](T sb, T pv, T cv, T mv, T& pb, T& cb, T& mb) {
    const int k = minmod_pick(pv - cv, cv - mv);
    pb = pb + (k == 1 ? sb : T(0));
    cb = cb + (k == 1 ? -sb : (k == 2 ? sb : T(0)));
    mb = mb + (k == 2 ? -sb : T(0));
  };
  {  // the depth slope: the forward's choice from dh_of
    const T sb = T(0.5) * (bR.h - bL.h);
    const int k = minmod_pick(dh_of(p, c), dh_of(c, m));
    bp.h = bp.h + (k == 1 ? sb : T(0));
    bc.h = bc.h + (k == 1 ? -sb : (k == 2 ? sb : T(0)));
    bm.h = bm.h + (k == 2 ? -sb : T(0));
  }
  if (m.h > dry_eps && c.h > dry_eps && p.h > dry_eps) {
    slope(T(0.5) * (bR.eta - bL.eta), p.eta, c.eta, m.eta, bp.eta, bc.eta,
          bm.eta);
    slope(T(0.5) * (bR.un - bL.un), p.un, c.un, m.un, bp.un, bc.un, bm.un);
    slope(T(0.5) * (bR.ut - bL.ut), p.ut, c.ut, m.ut, bp.ut, bc.ut, bm.ut);
  }
}

// partial derivatives of desing(h, q) (the forward formula's branch)
template <typename T>
__device__ __forceinline__ void desing_partials(T h, T q, T delta, T& dh,
                                                T& dq) {
  const T h4 = h * h * h * h;
  const T d4 = delta * delta * delta * delta;
  const bool big = h4 > d4;
  const T D4 = h4 + (big ? h4 : d4);
  const T s = sqrt(D4);
  const T f = sqrt(T(2)) * h * q / s;
  const T dD4 = (big ? T(8) : T(4)) * h * h * h;
  dq = sqrt(T(2)) * h / s;
  dh = sqrt(T(2)) * q / s - T(0.5) * f * dD4 / D4;
}

template <typename T>
__device__ __forceinline__ void add_bar(PrimBar<T>& t, const PrimBar<T>& b) {
  t.h = t.h + b.h;
  t.un = t.un + b.un;
  t.ut = t.ut + b.ut;
  t.eta = t.eta + b.eta;
}

// adds b to the accumulators of the line positions it belongs to: j itself
// (b0) and its mirrored ghosts gl, gh (bl, bh; equal to j0 when absent)
template <typename T>
__device__ __forceinline__ void to_positions(int pos, const PrimBar<T>& b,
                                             int j0, int gl, int gh,
                                             PrimBar<T>& b0, PrimBar<T>& bl,
                                             PrimBar<T>& bh) {
  if (pos == j0) add_bar(b0, b);
  if (gl != j0 && pos == gl) add_bar(bl, b);
  if (gh != j0 && pos == gh) add_bar(bh, b);
}

template <typename T, int DIR>
__global__ void __launch_bounds__(kBlock)
    k_adj_fv(AdjGeom G, const T* __restrict__ h, const T* __restrict__ q1,
             const T* __restrict__ q2, const T* __restrict__ H,
             const T* __restrict__ hs_out, const T* __restrict__ lhs,
             const T* __restrict__ lq1s, const T* __restrict__ lq2s,
             T* __restrict__ lh, T* __restrict__ lq1, T* __restrict__ lq2,
             T* __restrict__ lH) {
  constexpr bool XD = DIR == 1;
  const int nx = G.nx, ny = G.ny;
  const int n = xcd_bid() * kBlock + (int)threadIdx.x;
  if (n >= nx * ny) return;
  const int jx = n % nx, jy = n / nx;
  const int len = XD ? nx : ny, j0 = XD ? jx : jy;
  const T dry_eps = (T)G.dry_eps, g = (T)G.g, delta = (T)G.delta;
  const T dt = (T)(*G.dtp);
  const T fac = -dt / (XD ? (T)G.dx : (T)G.dy);
  // positions beyond one reflection (reached only on lines of 2 or 3 cells)
  // feed no cotangent; they are clamped to stay inside the grid
  auto prim_at = [&](int c) {
    c = min(max(c, -len), 2 * len - 1);
    return prim(XD ? load_cell(h, q1, q2, H, c, jy, nx, ny, false)
                   : load_cell(h, q1, q2, H, jx, c, nx, ny, false),
                XD, delta, false);
  };
  // adjoint weights of the direction's flux components (h, normal, tangent)
  // of cell c along the line; zero outside the grid
  auto weights = [&](int c, T w[3]) {
    w[0] = w[1] = w[2] = T(0);
    if (c < 0 || c >= len) return;
    const int m = XD ? jy * nx + c : c * nx + jx;
    const T hv = Store<T>::depth(hs_out[m], H[m]);
    const bool wet = hv > dry_eps;
    w[0] = hv > T(0) ? fac * lhs[m] : T(0);
    const T w1 = wet ? fac * lq1s[m] : T(0), w2 = wet ? fac * lq2s[m] : T(0);
    w[1] = XD ? w1 : w2;
    w[2] = XD ? w2 : w1;
  };
  // positions whose primitive values are j's: j itself and the ghosts
  // mirrored onto it (-1 - j at the low wall, 2 len - 1 - j at the high one)
  const int gl = j0 <= 1 ? -1 - j0 : j0;
  const int gh = j0 >= len - 2 ? 2 * len - 1 - j0 : j0;
  const int lo = max(min(gl, j0) - 1, -1), hi = min(max(gh, j0) + 1, len);
  PrimBar<T> b0{T(0), T(0), T(0), T(0)}, bl = b0, bh = b0;
  Prim<T> Pm2 = prim_at(lo - 3), Pm = prim_at(lo - 2), P0 = prim_at(lo - 1);
  Face<T> Lprev, Rprev;
  FaceBar<T> bLprev, bRprev;
  zero(bLprev);
  zero(bRprev);
  T h0bprev = T(0);
#pragma unroll 1
  for (int c = lo - 1; c <= hi + 1; ++c) {
    const Prim<T> Pp = prim_at(c + 1);
    Face<T> Lc, Rc;
    reconstruct(Pm, P0, Pp, dry_eps, Lc, Rc);
    FaceBar<T> bLc, bRc;
    zero(bLc);
    zero(bRc);
    T h0b = T(0);
    if (c >= lo && c >= 0 && c <= len) {  // edge (c-1 | c)
      T wl[3], wr[3];
      weights(c - 1, wl);
      weights(c, wr);
      pvm_rev(Rprev, Lc, g, dry_eps, wl, wr, bRprev, bLc);
    }
    if (c >= lo && c <= hi && c >= 0 && c < len) {  // volume term of c
      T w[3];
      weights(c, w);
      interior_rev(Lc, Rc, P0.h, g, w, bLc, bRc, h0b);
    }
    if (c - 1 >= lo && c - 1 <= hi) {  // reconstruction of c-1 is complete
      PrimBar<T> bm{T(0), T(0), T(0), T(0)}, bc = bm, bp = bm;
      bc.h = h0bprev;
      reconstruct_rev(Pm2, Pm, P0, dry_eps, Lprev, Rprev, bLprev, bRprev, bm,
                      bc, bp);
      to_positions(c - 2, bm, j0, gl, gh, b0, bl, bh);
      to_positions(c - 1, bc, j0, gl, gh, b0, bl, bh);
      to_positions(c, bp, j0, gl, gh, b0, bl, bh);
    }
    Pm2 = Pm;
    Pm = P0;
    P0 = Pp;
    Lprev = Lc;
    Rprev = Rc;
    bLprev = bLc;
    bRprev = bRc;
    h0bprev = h0b;
  }
  // a ghost's normal velocity is desing(h, -qn) = -desing(h, qn)
  PrimBar<T> b = b0;
  bl.un = -bl.un;
  bh.un = -bh.un;
  if (gl != j0) add_bar(b, bl);
  if (gh != j0) add_bar(b, bh);
  // primitives of j: un = desing(h, qn), ut = desing(h, qt), eta = h - H
  const T hj = Store<T>::depth(h[n], H[n]), qn = XD ? q1[n] : q2[n],
          qt = XD ? q2[n] : q1[n];
  T dhn, dqn, dht, dqt;
  desing_partials(hj, qn, delta, dhn, dqn);
  desing_partials(hj, qt, delta, dht, dqt);
  E ah = (E)b.h + (E)b.eta + (E)(dhn * b.un) + (E)(dht * b.ut);
  E an = (E)(dqn * b.un), at = (E)(dqt * b.ut);
  if (XD) {  // d out_j / d U_j contains the identity once
    const T hv = Store<T>::depth(hs_out[n], H[n]);
    const bool wet = hv > dry_eps;
    ah = ah + (hv > T(0) ? (E)lhs[n] : 0.0);
    an = an + (wet ? (E)lq1s[n] : 0.0);
    at = at + (wet ? (E)lq2s[n] : 0.0);
  }
  lh[n] = (T)((E)lh[n] + ah);
  lq1[n] = (T)((E)lq1[n] + (XD ? an : at));
  lq2[n] = (T)((E)lq2[n] + (XD ? at : an));
  lH[n] = (T)((E)lH[n] - (E)b.eta);
}

// Manning friction on the stage's finite-volume result (the forward's
// fv_finish): in wet cells q_out = q / den, den = 1 + dt fric |u| / h^(4/3),
// |u| from the desingularised velocities of (h, q).  Given the adjoint of
// q_out in (lqa, lqb), replaces it by the adjoint of the pre-friction q and
// adds the friction's share to the adjoint of h (|u|' = 0 at |u| = 0).
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_adj_friction(AdjGeom G, T fric, const T* __restrict__ hs,
                   const T* __restrict__ H, const T* __restrict__ qa,
                   const T* __restrict__ qb, T* __restrict__ lqa,
                   T* __restrict__ lqb, T* __restrict__ lh) {
  const int n = xcd_bid() * kBlock + (int)threadIdx.x;
  if (n >= G.nx * G.ny) return;
  const T h = Store<T>::depth(hs[n], H[n]);
  if (h <= (T)G.dry_eps) return;  // dry: q = 0, no friction
  const T dt = (T)(*G.dtp), delta = (T)G.delta, K = dt * fric;
  const T a = qa[n], b = qb[n];
  const T u = desing(h, a, delta), v = desing(h, b, delta);
  const T sp = sqrt(u * u + v * v);
  const T h43 = h * cbrt(h);
  const T den = T(1) + K * sp / h43;
  const T la = lqa[n], lb = lqb[n];
  const T lden = -(la * a + lb * b) / (den * den);
  T lan = la / den, lbn = lb / den;
  T lhn = -lden * K * sp * (T(4) / T(3)) / (h43 * h);
  if (sp > T(0)) {
    const T ls = lden * K / h43;
    T dh, dq;
    desing_partials(h, a, delta, dh, dq);
    lan = lan + ls * (u / sp) * dq;
    lhn = lhn + ls * (u / sp) * dh;
    desing_partials(h, b, delta, dh, dq);
    lbn = lbn + ls * (v / sp) * dq;
    lhn = lhn + ls * (v / sp) * dh;
  }
  lqa[n] = lan;
  lqb[n] = lbn;
  lh[n] = (T)((E)lh[n] + (E)lhn);
}

// ---------------------------------------------------------------------------
// correction (eq. 36, 41).  q = q* + dt T(p; h*, H) (zero where dry),
// w = w_in + dt desing(h_c, p) at the corners.  Per cell i with the corner
// pressures pSW, pSE, pNW, pNE and zx, zy the central differences of
// zeta = h* - 2H (eq. 36):
//   q1 += dt/2 (TN + TS),  TN + TS = -hc/(2dx) (pNE - pNW + pSE - pSW)
//                                    - zx/4 (pNE + pNW + pSE + pSW),
//   q2 += dt/2 (TE + TW),  TE + TW = -hc/(2dy) (pNE - pSE + pNW - pSW)
//                                    - zy/4 (same sum).
// Both are linear in p and in (hc, zx, zy), so their adjoints are written
// out: with a = dt/2 lq1_i, b = dt/2 lq2_i (0 where dry),
//   k_adj_correct_p: pbar_c = sum over the cells around c of
//     a (+-hc/(2dx) - zx/4) + b (+-hc/(2dy) - zy/4)    (+ west/south of c)
//     + dt lw_c d desing/dp                              (one per corner)
//   k_adj_correct_h: lhs_j += the hc, zeta (through the zx, zy of the cells
//     beside j, mirrored at walls) and corner-mean (w) terms, lH_j -= 2 x
//     the zeta terms; lqs_j = lq_j where wet             (one per cell)
// ---------------------------------------------------------------------------

// the positions a in [lo, hi] with mirror(a, n) == j (n >= 2, so one
// reflection covers [-2, n + 1]); returns their count
__device__ __forceinline__ int mirror_preimages(int j, int lo, int hi, int n,
                                                int a[3]) {
  int cnt = 0;
  const int cand[3] = {j, -1 - j, 2 * n - 1 - j};
#pragma unroll
  for (int t = 0; t < 3; ++t)
    if (cand[t] >= lo && cand[t] <= hi) a[cnt++] = cand[t];
  return cnt;
}

// forward values of cell q from its stored depth value (Store): the depth
// and zeta = h - 2H, in the arithmetic E of the adjoint sums (FP32 bulk:
// from s = h - max(H, 0))
template <typename T>
__device__ __forceinline__ E depth_e(const T* __restrict__ s,
                                     const T* __restrict__ H, int q) {
  if constexpr (Store<T>::kEta)
    return (E)s[q] + (H[q] > T(0) ? (E)H[q] : E(0));
  else
    return (E)s[q];
}
template <typename T>
__device__ __forceinline__ E zeta_e(const T* __restrict__ s,
                                    const T* __restrict__ H, int q) {
  if constexpr (Store<T>::kEta)
    return H[q] > T(0) ? (E)s[q] - (E)H[q] : (E)s[q] - E(2) * (E)H[q];
  else
    return (E)s[q] - E(2) * (E)H[q];
}

// per cell of the correction: a, b (dt/2 times the adjoint of q1, q2; zero
// where dry), hc and the zeta differences zx, zy (undivided by 2dx, 2dy)
template <typename T>
struct CorrCell {
  E a, b, hc, zx, zy;
};

template <typename T>
__device__ __forceinline__ CorrCell<T> corr_cell(const AdjGeom& G,
                                                 const T* __restrict__ hs,
                                                 const T* __restrict__ H,
                                                 const T* __restrict__ lq1,
                                                 const T* __restrict__ lq2,
                                                 E dt, int i, int j) {
  const int nx = G.nx, ny = G.ny, m = j * nx + i;
  auto zeta = [&](int ii, int jj) {
    return zeta_e(hs, H, mirror(jj, ny) * nx + mirror(ii, nx));
  };
  CorrCell<T> c;
  c.hc = depth_e(hs, H, m);
  const bool wet = !(Store<T>::depth(hs[m], H[m]) <= (T)G.dry_eps);
  c.a = wet ? E(0.5) * dt * (E)lq1[m] : 0.0;
  c.b = wet ? E(0.5) * dt * (E)lq2[m] : 0.0;
  c.zx = zeta(i + 1, j) - zeta(i - 1, j);
  c.zy = zeta(i, j + 1) - zeta(i, j - 1);
  return c;
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_adj_correct_p(AdjGeom G, const T* __restrict__ hs,
                    const T* __restrict__ H, const double* __restrict__ p,
                    const T* __restrict__ lq1, const T* __restrict__ lq2,
                    const T* __restrict__ lw, T* __restrict__ pbar) {
  const int nx = G.nx, ny = G.ny, ncx = nx + 1;
  const int c = xcd_bid() * kBlock + (int)threadIdx.x;
  if (c >= ncx * (ny + 1)) return;
  const int k = c % ncx, l = c / ncx;
  const E dx = G.dx, dy = G.dy, dt = *G.dtp;
  E acc = 0.0;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int i = k - 1 + (s & 1), j = l - 1 + (s >> 1);
    if (i < 0 || i >= nx || j < 0 || j >= ny) continue;
    const CorrCell<T> q = corr_cell<T>(G, hs, H, lq1, lq2, dt, i, j);
    // the corner is east of cell i for s & 1 == 0 (k = i + 1), north for
    // s >> 1 == 0 (l = j + 1)
    const E sx = (s & 1) ? E(1) : E(-1), sy = (s >> 1) ? E(1) : E(-1);
    acc = acc + q.a * (sx * q.hc / (E(2) * dx) - q.zx / (E(8) * dx)) +
          q.b * (sy * q.hc / (E(2) * dy) - q.zy / (E(8) * dy));
  }
  // w_c = w_in + dt desing(mean of the corner's cells, p_c)
  auto hcell = [&](int i, int j) {
    return depth_e(hs, H, mirror(j, ny) * nx + mirror(i, nx));
  };
  const E hm = E(0.25) * (hcell(k - 1, l - 1) + hcell(k, l - 1) +
                          hcell(k - 1, l) + hcell(k, l));
  E dh, dq;
  desing_partials<E>(hm, (E)(T)p[c], (E)G.delta, dh, dq);
  acc = acc + dt * dq * (E)lw[c];
  pbar[c] = (T)acc;
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_adj_correct_h(AdjGeom G, const T* __restrict__ hs,
                    const T* __restrict__ H, const double* __restrict__ p,
                    const T* __restrict__ lq1, const T* __restrict__ lq2,
                    const T* __restrict__ lw, T* __restrict__ lhs,
                    T* __restrict__ lH, T* __restrict__ lq1s,
                    T* __restrict__ lq2s) {
  const int nx = G.nx, ny = G.ny, ncx = nx + 1;
  const int n = xcd_bid() * kBlock + (int)threadIdx.x;
  if (n >= nx * ny) return;
  const int jx = n % nx, jy = n / nx;
  const E dx = G.dx, dy = G.dy, dt = *G.dtp;
  auto pc = [&](int k, int l) { return (E)(T)p[l * ncx + k]; };
  E ah = 0.0, az = 0.0;
  {  // hc of cell j itself
    const CorrCell<T> q = corr_cell<T>(G, hs, H, lq1, lq2, dt, jx, jy);
    const E pSW = pc(jx, jy), pSE = pc(jx + 1, jy);
    const E pNW = pc(jx, jy + 1), pNE = pc(jx + 1, jy + 1);
    ah = ah - q.a * ((pNE - pNW) + (pSE - pSW)) / (E(2) * dx) -
         q.b * ((pNE - pSE) + (pNW - pSW)) / (E(2) * dy);
  }
  // zeta of j in zx of the cells i with mirror(i +- 1) == jx (same row),
  // and in zy of the cells with mirror(i +- 1) == jy (same column):
  // d(TN + TS)/d zx = -(sum of the cell's corner pressures) / (4 2dx)
  auto psum = [&](int i, int j) {
    return pc(i, j) + pc(i + 1, j) + pc(i, j + 1) + pc(i + 1, j + 1);
  };
  int t[3];
  int nt = mirror_preimages(jx, 1, nx, nx, t);  // i + 1 reads j
  for (int u = 0; u < nt; ++u) {
    const int i = t[u] - 1;
    const CorrCell<T> q = corr_cell<T>(G, hs, H, lq1, lq2, dt, i, jy);
    az = az - q.a * psum(i, jy) / (E(8) * dx);
  }
  nt = mirror_preimages(jx, -1, nx - 2, nx, t);  // i - 1 reads j
  for (int u = 0; u < nt; ++u) {
    const int i = t[u] + 1;
    const CorrCell<T> q = corr_cell<T>(G, hs, H, lq1, lq2, dt, i, jy);
    az = az + q.a * psum(i, jy) / (E(8) * dx);
  }
  nt = mirror_preimages(jy, 1, ny, ny, t);
  for (int u = 0; u < nt; ++u) {
    const int j = t[u] - 1;
    const CorrCell<T> q = corr_cell<T>(G, hs, H, lq1, lq2, dt, jx, j);
    az = az - q.b * psum(jx, j) / (E(8) * dy);
  }
  nt = mirror_preimages(jy, -1, ny - 2, ny, t);
  for (int u = 0; u < nt; ++u) {
    const int j = t[u] + 1;
    const CorrCell<T> q = corr_cell<T>(G, hs, H, lq1, lq2, dt, jx, j);
    az = az + q.b * psum(jx, j) / (E(8) * dy);
  }
  // corner means: j is 1 or 2 (at a wall) of the 4 mirrored cells per axis
  auto hcell = [&](int i, int j) {
    return depth_e(hs, H, mirror(j, ny) * nx + mirror(i, nx));
  };
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int k = jx + (s & 1), l = jy + (s >> 1);
    const int mx = (mirror(k - 1, nx) == jx) + (mirror(k, nx) == jx);
    const int my = (mirror(l - 1, ny) == jy) + (mirror(l, ny) == jy);
    const E hm = E(0.25) * (hcell(k - 1, l - 1) + hcell(k, l - 1) +
                            hcell(k - 1, l) + hcell(k, l));
    E dh, dq;
    desing_partials<E>(hm, pc(k, l), (E)G.delta, dh, dq);
    ah = ah + E(0.25) * E(mx * my) * dt * dh * (E)lw[l * ncx + k];
  }
  // zeta = h - 2H
  lhs[n] = (T)((E)lhs[n] + ah + az);
  lH[n] = (T)((E)lH[n] - E(2) * az);
  const bool wet = Store<T>::depth(hs[n], H[n]) > (T)G.dry_eps;
  lq1s[n] = wet ? lq1[n] : T(0);
  lq2s[n] = wet ? lq2[n] : T(0);
}

// ---------------------------------------------------------------------------
// pressure system.  R_c(U) = rhs_c - (A p)_c at fixed p; the adjoint of U
// gains sum_c mu_c dR_c/dU.  Every row is a polynomial in the cells it reads
// (closed-form 5-point coefficients, eq. 43 in 2D), so it is differentiated
// in reverse: one pass per corner carries mu_c back to the 15 pair averages
// of the row (kRowBars, below), and one pass per cell gathers them.
//   corner pass: hc = (h_SW + h_SE + h_NW + h_NE)/4; hE, hW, hN, hS and
//     XE, XW, YN, YS the side averages of h and of the central zeta
//     differences X, Y (zeta = h - 2H); sx, sy the zeta differences across
//     the corner; q1E, q1W, q2N, q2S the side averages of the discharges.
//   cell pass: cell j sits at one of the 4 positions of each corner around
//     it, and the X, Y of its neighbours read its zeta; at the walls the
//     mirrored ghost positions fold onto j (discharge sign flipped across).
// dR_c/dw_c goes straight to lw_c in the corner pass.
// ---------------------------------------------------------------------------
enum RowBar {
  kBhc, kBhE, kBhW, kBhN, kBhS, kBXE, kBXW, kBYN, kBYS, kBsx, kBsy,
  kBq1E, kBq1W, kBq2N, kBq2S, kRowBars
};

template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_adj_row_bars(AdjGeom G, const T* __restrict__ hs,
                   const T* __restrict__ q1s, const T* __restrict__ q2s,
                   const T* __restrict__ H, const T* __restrict__ ws,
                   const double* __restrict__ p, const double* __restrict__ mu,
                   T* __restrict__ rb, T* __restrict__ lw) {
  const int nx = G.nx, ny = G.ny, ncx = nx + 1;
  const long ncorn = (long)ncx * (ny + 1);
  const int c = xcd_bid() * kBlock + (int)threadIdx.x;
  if (c >= ncorn) return;
  const int k = c % ncx, l = c / ncx;
  auto zeta = [&](int i, int j) {
    return zeta_e(hs, H, mirror(j, ny) * nx + mirror(i, nx));
  };
  // SW, SE, NW, NE cells of the corner (mirrored; discharges flip sign
  // across the wall they are mirrored over)
  E hh[4], zz[4], XX[4], YY[4], a1[4], a2[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int i = k - 1 + (s & 1), j = l - 1 + (s >> 1);
    const int mi = mirror(i, nx), mj = mirror(j, ny), m = mj * nx + mi;
    hh[s] = depth_e(hs, H, m);
    zz[s] = zeta_e(hs, H, m);
    a1[s] = mi != i ? -(E)q1s[m] : (E)q1s[m];
    a2[s] = mj != j ? -(E)q2s[m] : (E)q2s[m];
    XX[s] = (zeta(i + 1, j) - zeta(i - 1, j)) / E(2);
    YY[s] = (zeta(i, j + 1) - zeta(i, j - 1)) / E(2);
  }
  const int SW = 0, SE = 1, NW = 2, NE = 3;
  const E hc = E(0.25) * (hh[SW] + hh[SE] + hh[NW] + hh[NE]);
  const E hE = E(0.5) * (hh[SE] + hh[NE]), hW = E(0.5) * (hh[SW] + hh[NW]);
  const E hN = E(0.5) * (hh[NW] + hh[NE]), hS = E(0.5) * (hh[SW] + hh[SE]);
  const E XE = E(0.5) * (XX[SE] + XX[NE]), XW = E(0.5) * (XX[SW] + XX[NW]);
  const E YN = E(0.5) * (YY[NW] + YY[NE]), YS = E(0.5) * (YY[SW] + YY[SE]);
  const E sx = E(0.5) * (zz[SE] + zz[NE]) - E(0.5) * (zz[SW] + zz[NW]);
  const E sy = E(0.5) * (zz[NW] + zz[NE]) - E(0.5) * (zz[SW] + zz[SE]);
  const E q1E = E(0.5) * (a1[SE] + a1[NE]), q1W = E(0.5) * (a1[SW] + a1[NW]);
  const E q2N = E(0.5) * (a2[NW] + a2[NE]), q2S = E(0.5) * (a2[SW] + a2[SE]);
  const E dx = G.dx, dy = G.dy, dx2 = dx * dx, dy2 = dy * dy;
  const E Ap = E(2) * hc + sx, Am = E(2) * hc - sx;  // x factors of the row
  const E Bp = E(2) * hc + sy, Bm = E(2) * hc - sy;  // y factors
  // neighbour pressures the folded row multiplies: at a wall the outward
  // coefficient is added to the inward one
  const E p0 = p[c];
  const E PE = k < nx ? p[c + 1] : p[c - 1], PW = k > 0 ? p[c - 1] : p[c + 1];
  const E PN = l < ny ? p[c + ncx] : p[c - ncx];
  const E PS = l > 0 ? p[c - ncx] : p[c + ncx];
  // R = rhs - (d p0 + e PE + w PW + n PN + s PS), rhs = -(4/dt) Bs
  const E m = mu[c];
  const E db = -m * p0, eb = -m * PE, wb = -m * PW, nb = -m * PN,
          sb = -m * PS;
  const E Bsb = -(E(4) / *G.dtp) * m;
  const E Apb = (db * (XW + E(2) * hW) + wb * (XW - E(2) * hW)) / dx2 -
                Bsb * q1W / dx;
  const E Amb = -(db * (XE - E(2) * hE) + eb * (XE + E(2) * hE)) / dx2 +
                Bsb * q1E / dx;
  const E Bpb = (db * (YS + E(2) * hS) + sb * (YS - E(2) * hS)) / dy2 -
                Bsb * q2S / dy;
  const E Bmb = -(db * (YN - E(2) * hN) + nb * (YN + E(2) * hN)) / dy2 +
                Bsb * q2N / dy;
  const E wc = (E)ws[c];
  T* o = rb + c;
  o[kBhc * ncorn] = (T)(E(2) * (Apb + Amb + Bpb + Bmb) + E(4) * wc * Bsb);
  o[kBhE * ncorn] = (T)(E(2) * Am * (db - eb) / dx2);
  o[kBhW * ncorn] = (T)(E(2) * Ap * (db - wb) / dx2);
  o[kBhN * ncorn] = (T)(E(2) * Bm * (db - nb) / dy2);
  o[kBhS * ncorn] = (T)(E(2) * Bp * (db - sb) / dy2);
  o[kBXE * ncorn] = (T)(-Am * (db + eb) / dx2);
  o[kBXW * ncorn] = (T)(Ap * (db + wb) / dx2);
  o[kBYN * ncorn] = (T)(-Bm * (db + nb) / dy2);
  o[kBYS * ncorn] = (T)(Bp * (db + sb) / dy2);
  o[kBsx * ncorn] = (T)(Apb - Amb);
  o[kBsy * ncorn] = (T)(Bpb - Bmb);
  o[kBq1E * ncorn] = (T)(Bsb * Am / dx);
  o[kBq1W * ncorn] = (T)(-Bsb * Ap / dx);
  o[kBq2N * ncorn] = (T)(Bsb * Bm / dy);
  o[kBq2S * ncorn] = (T)(-Bsb * Bp / dy);
  lw[c] = (T)((E)lw[c] + E(4) * hc * Bsb);
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_adj_row_gather(AdjGeom G, const T* __restrict__ rb,
                     T* __restrict__ lhs, T* __restrict__ lq1s,
                     T* __restrict__ lq2s, T* __restrict__ lH) {
  const int nx = G.nx, ny = G.ny, ncx = nx + 1;
  const long ncorn = (long)ncx * (ny + 1);
  const int n = xcd_bid() * kBlock + (int)threadIdx.x;
  if (n >= nx * ny) return;
  const int jx = n % nx, jy = n / nx;
  auto bar = [&](int q, int k, int l) {
    return (E)rb[q * ncorn + l * ncx + k];
  };
  // sums over the corners around the (unmirrored) cell position (u, v):
  // the corner at (u, .) has the cell on its east side, at (u + 1, .) west;
  // at (., v) north, at (., v + 1) south
  auto xsum = [&](int u, int v) {  // X of the position, one half per side
    E s = 0.0;
    for (int dk = 0; dk < 2; ++dk)
      for (int dl = 0; dl < 2; ++dl) {
        const int k = u + dk, l = v + dl;
        if (k < 0 || k > nx || l < 0 || l > ny) continue;
        s = s + E(0.5) * bar(dk == 0 ? kBXE : kBXW, k, l);
      }
    return s;
  };
  auto ysum = [&](int u, int v) {
    E s = 0.0;
    for (int dk = 0; dk < 2; ++dk)
      for (int dl = 0; dl < 2; ++dl) {
        const int k = u + dk, l = v + dl;
        if (k < 0 || k > nx || l < 0 || l > ny) continue;
        s = s + E(0.5) * bar(dl == 0 ? kBYN : kBYS, k, l);
      }
    return s;
  };
  int cx[3], cy[3];
  const int ncxs = mirror_preimages(jx, -1, nx, nx, cx);
  const int ncys = mirror_preimages(jy, -1, ny, ny, cy);
  E ah = 0.0, aq1 = 0.0, aq2 = 0.0, az = 0.0;
  // the cell at a corner position: its h, zeta and discharges
  for (int a = 0; a < ncxs; ++a)
    for (int b = 0; b < ncys; ++b) {
      const int u = cx[a], v = cy[b];
      E hb = 0.0, zb = 0.0, q1b = 0.0, q2b = 0.0;
      for (int dk = 0; dk < 2; ++dk)
        for (int dl = 0; dl < 2; ++dl) {
          const int k = u + dk, l = v + dl;
          if (k < 0 || k > nx || l < 0 || l > ny) continue;
          const bool east = dk == 0, north = dl == 0;
          hb = hb + (E(0.25) * bar(kBhc, k, l) +
                     E(0.5) * bar(east ? kBhE : kBhW, k, l) +
                     E(0.5) * bar(north ? kBhN : kBhS, k, l));
          zb = zb + E(0.5) * (east ? bar(kBsx, k, l) : -bar(kBsx, k, l)) +
               E(0.5) * (north ? bar(kBsy, k, l) : -bar(kBsy, k, l));
          q1b = q1b + E(0.5) * bar(east ? kBq1E : kBq1W, k, l);
          q2b = q2b + E(0.5) * bar(north ? kBq2N : kBq2S, k, l);
        }
      ah = ah + hb;
      az = az + zb;
      aq1 = u != jx ? aq1 - q1b : aq1 + q1b;
      aq2 = v != jy ? aq2 - q2b : aq2 + q2b;
    }
  // the cell's zeta in the central differences X, Y of the positions
  // beside it: X(u) = (zeta(u + 1) - zeta(u - 1)) / 2
  int t[3];
  int nt = mirror_preimages(jx, 0, nx + 1, nx, t);
  for (int a = 0; a < nt; ++a)
    for (int b = 0; b < ncys; ++b) az = az + E(0.5) * xsum(t[a] - 1, cy[b]);
  nt = mirror_preimages(jx, -2, nx - 1, nx, t);
  for (int a = 0; a < nt; ++a)
    for (int b = 0; b < ncys; ++b) az = az - E(0.5) * xsum(t[a] + 1, cy[b]);
  nt = mirror_preimages(jy, 0, ny + 1, ny, t);
  for (int b = 0; b < nt; ++b)
    for (int a = 0; a < ncxs; ++a) az = az + E(0.5) * ysum(cx[a], t[b] - 1);
  nt = mirror_preimages(jy, -2, ny - 1, ny, t);
  for (int b = 0; b < nt; ++b)
    for (int a = 0; a < ncxs; ++a) az = az - E(0.5) * ysum(cx[a], t[b] + 1);
  // zeta = h - 2H
  lhs[n] = (T)((E)lhs[n] + ah + az);
  lq1s[n] = (T)((E)lq1s[n] + aq1);
  lq2s[n] = (T)((E)lq2s[n] + aq2);
  lH[n] = (T)((E)lH[n] - E(2) * az);
}

// rows of A^T: (A^T mu)_c = diag_c mu_c + cW_{c+1} mu_{c+1} + cE_{c-1} mu_{c-1}
//                          + cS_{c+ncx} mu_{c+ncx} + cN_{c-ncx} mu_{c-ncx}
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_transpose_rows(int nx, int ny, const T* __restrict__ cE,
                     const T* __restrict__ cW, const T* __restrict__ cN,
                     const T* __restrict__ cS, T* __restrict__ tE,
                     T* __restrict__ tW, T* __restrict__ tN,
                     T* __restrict__ tS) {
  const int ncx = nx + 1;
  const int c = xcd_bid() * kBlock + (int)threadIdx.x;
  if (c >= ncx * (ny + 1)) return;
  const int k = c % ncx, l = c / ncx;
  tE[c] = k < nx ? cW[c + 1] : T(0);
  tW[c] = k > 0 ? cE[c - 1] : T(0);
  tN[c] = l < ny ? cS[c + ncx] : T(0);
  tS[c] = l > 0 ? cN[c - ncx] : T(0);
}

// max_c |b_c / diag_c| per workgroup (scale of the adjoint system)
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_scaled_max(int n, const T* __restrict__ b, const T* __restrict__ diag,
                 double* __restrict__ part) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  double v = 0.0;
  if (c < n) v = fabs((double)b[c] / (double)diag[c]);
  __shared__ double wmax[kBlock / 64];
  v = wave_max(v);
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = wmax[0];
    for (int w = 1; w < kBlock / 64; ++w)
      m = (wmax[w] > m || wmax[w] != wmax[w]) ? wmax[w] : m;
    part[blockIdx.x] = m;
  }
}

// ---------------------------------------------------------------------------
// elementwise pieces
// ---------------------------------------------------------------------------
// RK average U^{n+1} = (U^n + U^(2)) / 2: both receive half the adjoint
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_adj_half(long n, T* __restrict__ a, T* __restrict__ half_out) {
  const long i = (long)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const T v = T(0.5) * a[i];
  a[i] = v;
  half_out[i] = v;
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_axpy1(long n, const T* __restrict__ x, T* __restrict__ y) {
  const long i = (long)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) y[i] = y[i] + x[i];
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_copy(long n, const T* __restrict__ x, T* __restrict__ y) {
  const long i = (long)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) y[i] = x[i];
}

// gauge misfit after a forward step: res_g = h_g - target_g,
// J += 1/2 sum res_g^2 (one thread: a handful of gauges, in order)
template <typename T>
__global__ void k_gauge_misfit(int ng, const int* __restrict__ gauges,
                               const T* __restrict__ h,
                               const T* __restrict__ H,
                               const double* __restrict__ target,
                               double* __restrict__ res,
                               double* __restrict__ J) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double s = 0.0;
  for (int g = 0; g < ng; ++g) {
    double r = depth_e(h, H, gauges[g]) - target[g];
    res[g] = r;
    s += r * r;
  }
  *J += 0.5 * s;
}

// adjoint source of the misfit at one time level: lh_g += res_g
template <typename T>
__global__ void k_gauge_source(int ng, const int* __restrict__ gauges,
                               const double* __restrict__ res,
                               T* __restrict__ lh) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  for (int g = 0; g < ng; ++g) lh[gauges[g]] = lh[gauges[g]] + (T)res[g];
}

}  // namespace nh
