// adjoint.hpp -- device code of the adjoint (reverse) time step.
//
// The adjoint of one projection-correction stage is assembled from local
// transposed Jacobian products.  Each local Jacobian is evaluated exactly by
// running the forward formulas of kernels.hpp (fv_cell, assemble_row,
// correct_cell, correct_corner) on forward-mode dual numbers, seeded at one
// input; every branch (limiter, HLL speeds, wet/dry tests, clamps) takes the
// decision of the forward values.  The products are gathered: one thread per
// input cell or corner visits every output that reads it, so no two threads
// add into the same place and the result does not depend on scheduling.
//
// Pressure: the stage solves A(U) p = rhs(U).  With A^T mu = pbar (pbar the
// adjoint of p), the adjoint of U gains mu^T d(rhs - A p)/dU at fixed p.
#pragma once
#include "kernels.hpp"

namespace nh {

// value and N directional derivatives
template <typename T, int N>
struct Dual {
  T v;
  T d[N];
  __device__ __forceinline__ Dual() : v(T(0)) {
#pragma unroll
    for (int k = 0; k < N; ++k) d[k] = T(0);
  }
  __device__ __forceinline__ Dual(double x) : v((T)x) {
#pragma unroll
    for (int k = 0; k < N; ++k) d[k] = T(0);
  }
  __device__ __forceinline__ Dual(float x) : v((T)x) {
#pragma unroll
    for (int k = 0; k < N; ++k) d[k] = T(0);
  }
  __device__ __forceinline__ Dual(int x) : v((T)x) {
#pragma unroll
    for (int k = 0; k < N; ++k) d[k] = T(0);
  }

  friend __device__ __forceinline__ Dual operator+(const Dual& a,
                                                  const Dual& b) {
    Dual r;
    r.v = a.v + b.v;
#pragma unroll
    for (int k = 0; k < N; ++k) r.d[k] = a.d[k] + b.d[k];
    return r;
  }
  friend __device__ __forceinline__ Dual operator-(const Dual& a,
                                                  const Dual& b) {
    Dual r;
    r.v = a.v - b.v;
#pragma unroll
    for (int k = 0; k < N; ++k) r.d[k] = a.d[k] - b.d[k];
    return r;
  }
  friend __device__ __forceinline__ Dual operator-(const Dual& a) {
    Dual r;
    r.v = -a.v;
#pragma unroll
    for (int k = 0; k < N; ++k) r.d[k] = -a.d[k];
    return r;
  }
  friend __device__ __forceinline__ Dual operator*(const Dual& a,
                                                  const Dual& b) {
    Dual r;
    r.v = a.v * b.v;
#pragma unroll
    for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
    return r;
  }
  // the value is the forward's quotient (its branches see the same numbers);
  // the derivatives use one reciprocal
  friend __device__ __forceinline__ Dual operator/(const Dual& a,
                                                  const Dual& b) {
    Dual r;
    r.v = a.v / b.v;
    const T inv = T(1) / b.v;
#pragma unroll
    for (int k = 0; k < N; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) * inv;
    return r;
  }
  // at 0 (a dry face) the derivative is taken as 0: the forward run treats
  // such a face as dry, and its speeds do not move to first order
  friend __device__ __forceinline__ Dual sqrt(const Dual& a) {
    Dual r;
    r.v = sqrt(a.v);
    const T s = r.v > T(0) ? T(0.5) / r.v : T(0);
#pragma unroll
    for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * s;
    return r;
  }
  friend __device__ __forceinline__ Dual fabs(const Dual& a) {
    return a.v < T(0) ? -a : a;
  }
  friend __device__ __forceinline__ bool operator<(const Dual& a,
                                                  const Dual& b) {
    return a.v < b.v;
  }
  friend __device__ __forceinline__ bool operator>(const Dual& a,
                                                  const Dual& b) {
    return a.v > b.v;
  }
  friend __device__ __forceinline__ bool operator<=(const Dual& a,
                                                   const Dual& b) {
    return a.v <= b.v;
  }
  friend __device__ __forceinline__ bool operator>=(const Dual& a,
                                                   const Dual& b) {
    return a.v >= b.v;
  }
};

// Type of the local Jacobian evaluations: the finite-volume and pressure-row
// derivatives run in the bulk type (their cost dominates the adjoint step),
// the correction's in FP64; sums over outputs are always FP64.
using E = double;

// mirrored cells of the bulk arrays as FP64 duals; cell `seed` carries the
// directions dh (index ih), dq1 (iq1), dq2 (iq2), dH (iH) (-1: not seeded)
template <typename T, int N, typename V = E>
struct SeedLoader {
  const T *h, *q1, *q2, *H;
  int nx, ny, seed;
  int ih, iq1, iq2, iH;
  __device__ __forceinline__ Cell<Dual<V, N>> operator()(int i, int j) const {
    int mi = mirror(i, nx), mj = mirror(j, ny);
    int idx = mj * nx + mi;
    Cell<Dual<V, N>> c;
    c.h = Dual<V, N>((V)h[idx]);
    c.q1 = Dual<V, N>((V)q1[idx]);
    c.q2 = Dual<V, N>((V)q2[idx]);
    c.H = Dual<V, N>((V)H[idx]);
    if (idx == seed) {
      if (ih >= 0) c.h.d[ih] = V(1);
      if (iq1 >= 0) c.q1.d[iq1] = V(1);
      if (iq2 >= 0) c.q2.d[iq2] = V(1);
      if (iH >= 0) c.H.d[iH] = V(1);
    }
    if (mi != i) c.q1 = -c.q1;
    if (mj != j) c.q2 = -c.q2;
    return c;
  }
};

// corner pressures as FP64 duals (rounded to the bulk type first, as the
// forward correction reads them); corner `seed` carries direction 0
template <typename T, int N>
struct SeedPLoader {
  const double* p;
  int ncx, seed;
  __device__ __forceinline__ Dual<E, N> operator()(int k, int l) const {
    int idx = l * ncx + k;
    Dual<E, N> v((E)(T)p[idx]);
    if (idx == seed) v.d[0] = E(1);
    return v;
  }
};

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
// Per input cell j the pass slides along j's line over the cells j-2..j+2:
// their reconstructions, the 4 edges that read j and the 3 volume terms that
// read j, each once, on 4-direction dual numbers (dh, dq1, dq2, dH of j), and
//   lh_j += sum over those pieces of d(piece)/d(j) * (-dt/dx) * lambda(out),
// likewise q1, q2, H; the x pass adds j's own identity term.  hs_out (the
// stored h*) gives the forward's clamp and dry decisions.
// ---------------------------------------------------------------------------
template <typename T, int DIR>
__global__ void __launch_bounds__(kBlock)
    k_adj_fv(AdjGeom G, const T* __restrict__ h, const T* __restrict__ q1,
             const T* __restrict__ q2, const T* __restrict__ H,
             const T* __restrict__ hs_out, const T* __restrict__ lhs,
             const T* __restrict__ lq1s, const T* __restrict__ lq2s,
             T* __restrict__ lh, T* __restrict__ lq1, T* __restrict__ lq2,
             T* __restrict__ lH) {
  using D = Dual<T, 4>;
  constexpr bool XD = DIR == 1;
  const int nx = G.nx, ny = G.ny;
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= nx * ny) return;
  const int jx = n % nx, jy = n / nx;
  const int len = XD ? nx : ny, j0 = XD ? jx : jy;
  const T dry_eps = (T)G.dry_eps;
  const D g(G.g), delta(G.delta), de(G.dry_eps);
  const T dt = (T)(*G.dtp);
  const E fac = -(E)dt / (E)(XD ? (T)G.dx : (T)G.dy);
  SeedLoader<T, 4, T> ld{h, q1, q2, H, nx, ny, n, 0, 1, 2, 3};
  auto prim_at = [&](int c) {
    return prim(XD ? ld(c, jy) : ld(jx, c), XD, delta, false);
  };
  // adjoint weights of the direction's flux components (h, normal, tangent)
  // of cell c along the line
  auto weights = [&](int c, E w[3]) {
    const int m = XD ? jy * nx + c : c * nx + jx;
    const T hv = hs_out[m];
    const E wh = hv > T(0) ? (E)lhs[m] : 0.0;
    const bool wet = hv > dry_eps;
    const E w1 = wet ? (E)lq1s[m] : 0.0, w2 = wet ? (E)lq2s[m] : 0.0;
    w[0] = fac * wh;
    w[1] = fac * (XD ? w1 : w2);
    w[2] = fac * (XD ? w2 : w1);
  };
  E acc[4] = {0.0, 0.0, 0.0, 0.0};
  auto add = [&](const D f[3], const E w[3]) {
#pragma unroll
    for (int k = 0; k < 4; ++k)
      acc[k] = acc[k] + ((E)f[0].d[k] * w[0] + (E)f[1].d[k] * w[1] +
                         (E)f[2].d[k] * w[2]);
  };
  if (XD) {  // d out_j / d U_j contains the identity once
    const T hv = hs_out[n];
    const bool wet = hv > dry_eps;
    acc[0] = hv > T(0) ? (E)lhs[n] : 0.0;
    acc[1] = wet ? (E)lq1s[n] : 0.0;
    acc[2] = wet ? (E)lq2s[n] : 0.0;
  }
  Prim<D> Pm = prim_at(j0 - 3), P0 = prim_at(j0 - 2);
  Face<D> Rprev;
#pragma unroll 1
  for (int c = j0 - 2; c <= j0 + 2; ++c) {
    const Prim<D> Pp = prim_at(c + 1);
    Face<D> Lc, Rc;
    reconstruct(Pm, P0, Pp, de, Lc, Rc);
    const bool in_prev = c - 1 >= 0 && c - 1 < len, in_c = c >= 0 && c < len;
    if (c > j0 - 2 && (in_prev || in_c)) {  // edge (c-1 | c)
      D Dm[3], Dp[3];
      pvm(Rprev, Lc, g, de, Dm, Dp);
      E w[3];
      if (in_prev) {
        weights(c - 1, w);
        add(Dm, w);
      }
      if (in_c) {
        weights(c, w);
        add(Dp, w);
      }
    }
    if (c >= j0 - 1 && c <= j0 + 1 && in_c) {  // volume term of cell c
      D I[3];
      interior(Lc, Rc, P0.h, g, I);
      E w[3];
      weights(c, w);
      add(I, w);
    }
    Rprev = Rc;
    Pm = P0;
    P0 = Pp;
  }
  lh[n] = (T)((E)lh[n] + acc[0]);
  lq1[n] = (T)((E)lq1[n] + acc[1]);
  lq2[n] = (T)((E)lq2[n] + acc[2]);
  lH[n] = (T)((E)lH[n] + acc[3]);
}

// ---------------------------------------------------------------------------
// correction (eq. 36, 41).  q = q* + dt T(p; h*, H) (zero where dry),
// w = w_in + dt p / h_c.
//   k_adj_correct_p: pbar_c = sum over the cells i around corner c of
//     dq_i/dp_c lq_i + dw_c/dp_c lw_c                       (one per corner)
//   k_adj_correct_h: lhs_j += dq_i/dh*_j lq_i + dw_c/dh*_j lw_c, lH_j alike,
//     over the cells i in {j, its 4 neighbours} and the corners of j; and
//     lqs_j = lq_j where wet (0 where dry)                    (one per cell)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_adj_correct_p(AdjGeom G, const T* __restrict__ hs,
                    const T* __restrict__ H, const T* __restrict__ q1s,
                    const T* __restrict__ q2s, const T* __restrict__ ws,
                    const double* __restrict__ p, const T* __restrict__ lq1,
                    const T* __restrict__ lq2, const T* __restrict__ lw,
                    T* __restrict__ pbar) {
  using D = Dual<E, 1>;
  const int nx = G.nx, ny = G.ny, ncx = nx + 1;
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= ncx * (ny + 1)) return;
  const int k = c % ncx, l = c / ncx;
  const D dx(G.dx), dy(G.dy), de(G.dry_eps), delta(G.delta), dt(*G.dtp);
  SeedLoader<T, 1> ld{hs, q1s, q2s, H, nx, ny, -1, -1, -1, -1, -1};
  SeedPLoader<T, 1> pl{p, ncx, c};
  E acc = 0.0;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int i = k - 1 + (s & 1), j = l - 1 + (s >> 1);
    if (i < 0 || i >= nx || j < 0 || j >= ny) continue;
    const int m = j * nx + i;
    D qa(q1s[m]), qb(q2s[m]);
    correct_cell<D, false>(ld, pl, i, j, dx, dy, dt, de, qa, qb);
    acc = acc + (qa.d[0] * (E)lq1[m] + qb.d[0] * (E)lq2[m]);
  }
  D wv = correct_corner<D, false>(ld, k, l, D(ws[c]), pl(k, l), dt, delta);
  acc = acc + wv.d[0] * (E)lw[c];
  pbar[c] = (T)acc;
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_adj_correct_h(AdjGeom G, const T* __restrict__ hs,
                    const T* __restrict__ H, const T* __restrict__ q1s,
                    const T* __restrict__ q2s, const T* __restrict__ ws,
                    const double* __restrict__ p, const T* __restrict__ lq1,
                    const T* __restrict__ lq2, const T* __restrict__ lw,
                    T* __restrict__ lhs, T* __restrict__ lH,
                    T* __restrict__ lq1s, T* __restrict__ lq2s) {
  using D = Dual<E, 2>;
  const int nx = G.nx, ny = G.ny, ncx = nx + 1;
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= nx * ny) return;
  const int jx = n % nx, jy = n / nx;
  const D dx(G.dx), dy(G.dy), de(G.dry_eps), delta(G.delta), dt(*G.dtp);
  SeedLoader<T, 2> ld{hs, q1s, q2s, H, nx, ny, n, 0, -1, -1, 1};
  SeedPLoader<T, 2> pl{p, ncx, -1};
  E ah = 0.0, aH = 0.0;
  const int ox[5] = {0, -1, 1, 0, 0};
  const int oy[5] = {0, 0, 0, -1, 1};
#pragma unroll
  for (int o = 0; o < 5; ++o) {
    const int i = jx + ox[o], j = jy + oy[o];
    if (i < 0 || i >= nx || j < 0 || j >= ny) continue;
    const int m = j * nx + i;
    D qa(q1s[m]), qb(q2s[m]);
    correct_cell<D, false>(ld, pl, i, j, dx, dy, dt, de, qa, qb);
    ah = ah + (qa.d[0] * (E)lq1[m] + qb.d[0] * (E)lq2[m]);
    aH = aH + (qa.d[1] * (E)lq1[m] + qb.d[1] * (E)lq2[m]);
  }
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int k = jx + (s & 1), l = jy + (s >> 1);
    const int c = l * ncx + k;
    D wv = correct_corner<D, false>(ld, k, l, D(ws[c]), pl(k, l), dt, delta);
    ah = ah + wv.d[0] * (E)lw[c];
  }
  lhs[n] = (T)((E)lhs[n] + ah);
  lH[n] = (T)((E)lH[n] + aH);
  const bool wet = hs[n] > (T)G.dry_eps;
  lq1s[n] = wet ? lq1[n] : T(0);
  lq2s[n] = wet ? lq2[n] : T(0);
}

// ---------------------------------------------------------------------------
// pressure system.  R_c(U) = rhs_c - (A p)_c at fixed p.  Per cell j:
//   lhs_j += sum_c mu_c dR_c/dh*_j over the 12 corners whose row reads j,
// likewise q1*, q2*, H; per corner: lw_c += mu_c dR_c/dw*_c.
// ---------------------------------------------------------------------------
template <typename V>
__device__ __forceinline__ V row_residual(const V row[6], const double* p,
                                          int k, int l, int nx, int ny) {
  const int ncx = nx + 1, c = l * ncx + k;
  V Ap = row[0] * V(p[c]);
  if (k < nx) Ap = Ap + row[1] * V(p[c + 1]);
  if (k > 0) Ap = Ap + row[2] * V(p[c - 1]);
  if (l < ny) Ap = Ap + row[3] * V(p[c + ncx]);
  if (l > 0) Ap = Ap + row[4] * V(p[c - ncx]);
  return row[5] - Ap;
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_adj_assemble(AdjGeom G, const T* __restrict__ hs,
                   const T* __restrict__ q1s, const T* __restrict__ q2s,
                   const T* __restrict__ H, const T* __restrict__ ws,
                   const double* __restrict__ p, const double* __restrict__ mu,
                   T* __restrict__ lhs, T* __restrict__ lq1s,
                   T* __restrict__ lq2s, T* __restrict__ lH) {
  using D = Dual<T, 4>;
  const int nx = G.nx, ny = G.ny, ncx = nx + 1;
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= nx * ny) return;
  const int jx = n % nx, jy = n / nx;
  const D dx(G.dx), dy(G.dy), dt(*G.dtp);
  SeedLoader<T, 4, T> ld{hs, q1s, q2s, H, nx, ny, n, 0, 1, 2, 3};
  // corners (k, l) whose row reads cell (jx, jy): k in [jx-1, jx+2] on the
  // rows l = jy, jy+1, and k in [jx, jx+1] on the rows l = jy-1, jy+2
  const int ok[12] = {-1, 0, 1, 2, -1, 0, 1, 2, 0, 1, 0, 1};
  const int ol[12] = {0, 0, 0, 0, 1, 1, 1, 1, -1, -1, 2, 2};
  E acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int o = 0; o < 12; ++o) {
    const int k = jx + ok[o], l = jy + ol[o];
    if (k < 0 || k > nx || l < 0 || l > ny) continue;
    const int c = l * ncx + k;
    D row[6];
    assemble_row<D>(ld, k, l, nx, ny, dx, dy, D(ws[c]), dt, row);
    D R = row_residual<D>(row, p, k, l, nx, ny);
    const E m = mu[c];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = acc[q] + (E)R.d[q] * m;
  }
  lhs[n] = (T)((E)lhs[n] + acc[0]);
  lq1s[n] = (T)((E)lq1s[n] + acc[1]);
  lq2s[n] = (T)((E)lq2s[n] + acc[2]);
  lH[n] = (T)((E)lH[n] + acc[3]);
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_adj_assemble_w(AdjGeom G, const T* __restrict__ hs,
                     const T* __restrict__ q1s, const T* __restrict__ q2s,
                     const T* __restrict__ H, const T* __restrict__ ws,
                     const double* __restrict__ p,
                     const double* __restrict__ mu, T* __restrict__ lw) {
  using D = Dual<E, 1>;
  const int nx = G.nx, ny = G.ny, ncx = nx + 1;
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= ncx * (ny + 1)) return;
  const int k = c % ncx, l = c / ncx;
  const D dx(G.dx), dy(G.dy), dt(*G.dtp);
  SeedLoader<T, 1> ld{hs, q1s, q2s, H, nx, ny, -1, -1, -1, -1, -1};
  D wc(ws[c]);
  wc.d[0] = E(1);
  D row[6];
  assemble_row<D>(ld, k, l, nx, ny, dx, dy, wc, dt, row);
  D R = row_residual<D>(row, p, k, l, nx, ny);
  lw[c] = (T)((E)lw[c] + R.d[0] * mu[c]);
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
  const int c = blockIdx.x * kBlock + threadIdx.x;
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
                               const double* __restrict__ target,
                               double* __restrict__ res,
                               double* __restrict__ J) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double s = 0.0;
  for (int g = 0; g < ng; ++g) {
    double r = (double)h[gauges[g]] - target[g];
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
