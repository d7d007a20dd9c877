// kernels.hpp -- gfx950 device code of the non-hydrostatic shallow-water step
// (Escalante, Morales de Luna & Castro, arXiv 1706.04551).
//
// All kernels are templated on the storage/arithmetic type T of the bulk
// state (double, or float for the FP32-bulk mode).  The pressure solve always
// evaluates residuals, updates and its convergence measure in FP64.
//
// Layout: structure of arrays, row-major, x fastest.  Cells [ny][nx],
// corners [ny+1][nx+1] (1D: [nx+1]).  There are no ghost cells in memory:
// walls are applied by mirrored indexing (ghost -1 <-> cell 0, -2 <-> 1, the
// discharge normal to the wall changes sign, everything else is even).
//
// Every formula is evaluated in the same operation order as the plain
// statement of the scheme, so that FP64 results agree with a sequential
// evaluation to rounding.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nh {

constexpr int kBlock = 256;

// The workgroups of a launch go to the chip's 8 XCDs in turn (workgroup b
// to XCD b mod 8), and each XCD has an L2 of its own.  Numbering the work
// so that every XCD takes one contiguous run of it keeps the rows that
// neighbouring workgroups share (stencil halos, corner rows) in one L2
// instead of fetching them into two or three.  A bijection of [0, nb).
__device__ __forceinline__ int xcd_bid() {
  constexpr int kX = 8;
  const int b = (int)blockIdx.x, nb = (int)gridDim.x;
  const int q = nb / kX, r = nb % kX, x = b % kX;
  return x * q + min(x, r) + b / kX;
}

__device__ __forceinline__ int mirror(int i, int n) {
  return i < 0 ? -1 - i : (i >= n ? 2 * n - 1 - i : i);
}

// Boundary mask of a grid (the `open` field of the kernel arguments).  Open
// (outflow) sides, a bit each: homogeneous Neumann ghosts that copy the
// adjacent cell (Section 4.4).  Periodic directions (Section 4.4, item 1):
// the first and last cells of a line are neighbours, and the last corner of
// the line is its first (both are stored and hold the same values).  Every
// other side is a wall.
constexpr int kOpenW = 1, kOpenE = 2, kOpenS = 4, kOpenN = 8;
constexpr int kPerX = 16, kPerY = 32;

// the cell whose values position i of a line of n cells takes: its mirror
// image at a wall, the end cell itself at an open end, the cell one period
// away on a periodic line (i within two cells of the line)
__device__ __forceinline__ int ghost_src(int i, int n, bool open_lo,
                                         bool open_hi, bool per = false) {
  if (per) return i < 0 ? i + n : (i >= n ? i - n : i);
  if (i < 0) return open_lo ? 0 : -1 - i;
  if (i >= n) return open_hi ? n - 1 : 2 * n - 1 - i;
  return i;
}

// the stored corner that corner k of a periodic line of n cells is (corners
// 0 .. n are stored, n being 0 again; any k)
__device__ __forceinline__ int wrap_corner(int k, int n) {
  if (k < 0 || k > n) {
    k %= n;
    if (k < 0) k += n;
  }
  return k;
}

template <typename T>
__device__ __forceinline__ T tmax(T a, T b) { return a > b ? a : b; }
template <typename T>
__device__ __forceinline__ T tmin(T a, T b) { return a < b ? a : b; }

// minmod limiter of the MUSCL reconstruction (Section 4.1)
template <typename T>
__device__ __forceinline__ T minmod(T a, T b) {
  if (a > T(0) && b > T(0)) return tmin(a, b);
  if (a < T(0) && b < T(0)) return tmax(a, b);
  return T(0);
}

// desingularised velocity u = sqrt(2) h q / sqrt(h^4 + max(h^4, delta^4))
// (Section 4.5); also used for the division of the corner update by h_c.
template <typename T>
__device__ __forceinline__ T desing(T h, T q, T delta) {
  T h4 = h * h * h * h;
  T d4 = delta * delta * delta * delta;
  return sqrt(T(2)) * h * q / sqrt(h4 + tmax(h4, d4));
}

// What the depth arrays hold.  An FP64 grid stores the depth h.  An
// FP32-bulk grid stores s = h - R against the reference level R = max(H, 0):
// where the bed is below still water (H > 0) that is the surface elevation
// eta = h - H, so the slopes and edge jumps of eta (the well-balanced
// pressure terms, Section 4.1) are differences of stored values, where
// h - H formed in FP32 would keep only the digits h and H share (ulp(20 m)
// = 2e-6 m, against waves of centimetres); on land (H <= 0) it is the depth
// itself, so thin films on dry slopes keep their digits.  The update of s is
// the update of h (R does not change); a dry cell stores -R.
template <typename T>
struct Store;
template <>
struct Store<double> {
  static constexpr bool kEta = false;
  __device__ static double depth(double s, double H) { return s; }
  __device__ static double eta(double s, double H) { return s - H; }
  __device__ static double of_depth(double h, double H) { return h; }
};
template <>
struct Store<float> {
  static constexpr bool kEta = true;
  __device__ static float ref(float H) { return H > 0.f ? H : 0.f; }
  __device__ static float depth(float s, float H) { return s + ref(H); }
  __device__ static float eta(float s, float H) {
    return H > 0.f ? s : s - H;
  }
  __device__ static float of_depth(float h, float H) { return h - ref(H); }
};

// cell state with wall mirroring: depth h, surface elevation eta, the
// stored depth value s (h or eta, see Store), discharges, still-water depth
template <typename T>
struct Cell {
  T h, q1, q2, H, eta, s;
};

// zeta = 2 eta - h = h - 2H of a cell (the compact pressure scheme's
// combination, Appendix A): formed from h in FP64 as the oracle does, from
// the stored value in FP32 (one rounding instead of two cancelling ones)
template <typename T>
__device__ __forceinline__ T zeta_of(const Cell<T>& c) {
  if constexpr (Store<T>::kEta)
    return c.H > T(0) ? c.s - c.H : c.s - T(2) * c.H;
  else
    return c.h - T(2) * c.H;
}

template <typename T>
__device__ __forceinline__ Cell<T> load_cell(const T* __restrict__ h,
                                             const T* __restrict__ q1,
                                             const T* __restrict__ q2,
                                             const T* __restrict__ H, int i,
                                             int j, int nx, int ny,
                                             bool one_d, int open = 0) {
  const bool px = open & kPerX, py = !one_d && (open & kPerY);
  int mi = ghost_src(i, nx, open & kOpenW, open & kOpenE, px);
  int mj = one_d ? 0 : ghost_src(j, ny, open & kOpenS, open & kOpenN, py);
  int idx = mj * nx + mi;
  Cell<T> c;
  c.s = h[idx];
  c.H = H[idx];
  c.h = Store<T>::depth(c.s, c.H);
  c.eta = Store<T>::eta(c.s, c.H);
  c.q1 = q1[idx];
  c.q2 = one_d ? T(0) : q2[idx];
  // the normal discharge is odd across a wall, even across an open end and
  // across the seam of a periodic line
  if (mi != i && !px && !(open & (i < 0 ? kOpenW : kOpenE))) c.q1 = -c.q1;
  if (mj != j && !py && !(open & (j < 0 ? kOpenS : kOpenN))) c.q2 = -c.q2;
  return c;
}

// reconstructed state at one side of an edge, in edge-normal coordinates
template <typename T>
struct Face {
  T h, qn, qt, un, ut, eta, H;
};

// primitive values of a cell along a direction: n = normal discharge index
template <typename T>
struct Prim {
  T h, un, ut, eta;
  T s, R;  // FP32 bulk: stored depth value and reference level (Store)
};

// Depth difference b.h - a.h of two cells for the limiter.  In FP32 bulk it
// is formed from the stored values and the reference levels, each
// difference exact for nearby values and the sum rounded once: h = s + R
// formed in FP32 keeps only ulp(R) of the depth (4e-6 m on 50 m of water),
// more than the second differences the limiter compares on smooth waves
// over flat stretches of bed, where the choice would follow rounding noise.
template <typename T>
__device__ __forceinline__ T dh_of(const Prim<T>& b, const Prim<T>& a) {
  if constexpr (Store<T>::kEta)
    return (b.s - a.s) + (b.R - a.R);
  else
    return b.h - a.h;
}

template <typename T>
__device__ __forceinline__ Prim<T> prim(const Cell<T>& c, bool xdir, T delta,
                                        bool one_d) {
  Prim<T> p;
  p.h = c.h;
  T u = desing(c.h, c.q1, delta);
  T v = one_d ? T(0) : desing(c.h, c.q2, delta);
  p.un = xdir ? u : v;
  p.ut = xdir ? v : u;
  p.eta = c.eta;
  p.s = c.s;
  if constexpr (Store<T>::kEta)
    p.R = Store<T>::ref(c.H);
  else
    p.R = T(0);
  return p;
}

// MUSCL-minmod reconstruction of the middle cell c from its neighbours m, p:
// L = value at its minus-side edge, R = value at its plus-side edge.  Slopes
// of eta and of the velocities vanish next to a dry cell (Section 4.1, 4.5).
template <typename T>
__device__ __forceinline__ void reconstruct(const Prim<T>& m, const Prim<T>& c,
                                            const Prim<T>& p, T dry_eps,
                                            Face<T>& L, Face<T>& R) {
  T sh = minmod(dh_of(p, c), dh_of(c, m));
  T se = T(0), su = T(0), sv = T(0);
  if (m.h > dry_eps && c.h > dry_eps && p.h > dry_eps) {
    se = minmod(p.eta - c.eta, c.eta - m.eta);
    su = minmod(p.un - c.un, c.un - m.un);
    sv = minmod(p.ut - c.ut, c.ut - m.ut);
  }
  R.h = c.h + T(0.5) * sh;
  L.h = c.h - T(0.5) * sh;
  R.eta = c.eta + T(0.5) * se;
  L.eta = c.eta - T(0.5) * se;
  R.un = c.un + T(0.5) * su;
  L.un = c.un - T(0.5) * su;
  R.ut = c.ut + T(0.5) * sv;
  L.ut = c.ut - T(0.5) * sv;
  R.qn = R.h * R.un;
  L.qn = L.h * L.un;
  R.qt = R.h * R.ut;
  L.qt = L.h * L.ut;
  R.H = R.h - R.eta;
  L.H = L.h - L.eta;
}

// PVM fluctuations of eq. (18)-(19) with the A* matrix, HLL speeds and the
// emerging-bottom rule (Section 4.5).  Dm goes to the left cell, Dp to the
// right one; components (h, normal, tangential).
template <typename T>
__device__ __forceinline__ void pvm(const Face<T>& L, const Face<T>& R, T g,
                                    T dry_eps, T Dm[3], T Dp[3]) {
  Dm[0] = Dm[1] = Dm[2] = T(0);
  Dp[0] = Dp[1] = Dp[2] = T(0);
  if (L.h <= dry_eps && R.h <= dry_eps) return;
  T he = T(0.5) * (L.h + R.h);
  T sL = sqrt(L.h), sR = sqrt(R.h);
  T ue = (L.un * sL + R.un * sR) / (sL + sR);
  T ce = sqrt(g * he);
  T SL = tmin(ue - ce, L.un - sqrt(g * L.h));
  T SR = tmax(ue + ce, R.un + sqrt(g * R.h));
  if (!(SR - SL > T(0))) return;
  T a0 = (SR * fabs(SL) - SL * fabs(SR)) / (SR - SL);
  T a1 = (fabs(SR) - fabs(SL)) / (SR - SL);
  T deta = R.eta - L.eta;
  if (R.h <= dry_eps && L.eta < -R.H) deta = T(0);
  if (L.h <= dry_eps && R.eta < -L.H) deta = T(0);
  T Rv[3], dU[3];
  Rv[0] = R.qn - L.qn;
  Rv[1] = (R.qn * R.un - L.qn * L.un) + g * he * deta;
  Rv[2] = R.qn * R.ut - L.qn * L.ut;
  dU[0] = deta;
  dU[1] = R.qn - L.qn;
  dU[2] = R.qt - L.qt;
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    Dm[m] = T(0.5) * ((T(1) - a1) * Rv[m] - a0 * dU[m]);
    Dp[m] = T(0.5) * ((T(1) + a1) * Rv[m] + a0 * dU[m]);
  }
}

// volume term of eq. (22) in its mid-point form (eq. 30): the hydrostatic
// part 1/2 g (h-^2 - h+^2) - g h_i (H- - H+) equals g h_i (eta- - eta+) for
// the linear reconstruction; exact for the lake at rest.
template <typename T>
__device__ __forceinline__ void interior(const Face<T>& L, const Face<T>& R,
                                         T h0, T g, T I[3]) {
  I[0] = R.qn - L.qn;
  I[1] = (R.qn * R.un - L.qn * L.un) + g * h0 * (R.eta - L.eta);
  I[2] = R.qn * R.ut - L.qn * L.ut;
}

// -------------------------------------------------------------------------
// reductions of non-negative doubles: wavefront shuffle + LDS tree, then one
// 64-bit atomic max on the bit pattern (monotone for non-negative doubles)
// -------------------------------------------------------------------------
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    double o = __shfl_xor(v, off, 64);
    v = (o > v || o != o) ? o : v;
  }
  return v;
}

template <int B = kBlock>
__device__ __forceinline__ void block_max_to(double v,
                                             unsigned long long* dst) {
  __shared__ double part[B / 64];
  v = wave_max(v);
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) part[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = part[0];
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k)
      m = (part[k] > m || part[k] != part[k]) ? part[k] : m;
    if (m > 0.0 || m != m)
      atomicMax(dst, (unsigned long long)__double_as_longlong(m));
  }
}

__device__ __forceinline__ double block_sum(double v) {
  __shared__ double part[1024 / 64];  // any workgroup size
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) part[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += part[k];
  return s;
}

// -------------------------------------------------------------------------
// finite-volume stage: U* = V - dt (fluctuations + volume terms), eq. (20),
// (30); positivity clamp and dry discharge.
// -------------------------------------------------------------------------
// 2D stages run on tiles of kFvTX x kFvTY cells, one thread per cell
constexpr int kFvTX = 32, kFvTY = 8;
static_assert(kFvTX * kFvTY == kBlock, "one thread per tile cell");

template <typename T>
struct FvArgs {
  int nx, ny;
  T dx, dy, g, delta, dry_eps;
  const T *h, *q1, *q2, *H;
  const double* dtp;
  T *oh, *oq1, *oq2;
  double* clamped;
  T fric;  // g n^2 of the Manning friction law (Section 2); 0: none
  int open;  // open sides (kOpen*)
  __host__ __device__ int tiles_x() const { return (nx + kFvTX - 1) / kFvTX; }
  // 1D: one thread per cell; 2D: one workgroup per tile
  __host__ __device__ int nblocks() const {
    return ny == 1 ? (nx + kBlock - 1) / kBlock
                   : tiles_x() * ((ny + kFvTY - 1) / kFvTY);
  }
};

// loader of mirrored cells from the bulk arrays (walls by mirror images)
template <typename T, bool ONE_D>
struct CellLoader {
  const T *h, *q1, *q2, *H;
  int nx, ny;
  int open = 0;  // open sides (kOpen*)
  __device__ __forceinline__ Cell<T> operator()(int i, int j) const {
    return load_cell(h, q1, q2, H, i, j, nx, ny, ONE_D, open);
  }
};

// The finite-volume update of cell (i, j) (eq. 20-22, 30): the values
// h - dt (fx/dx + fy/dy), q1 - ..., q2 - ... before the positivity clamp.
// `ld(i, j)` returns the mirrored cell; V is the arithmetic type.  `parts`
// selects the x (1) and y (2) flux sums; a skipped part contributes zero.
template <typename V, bool ONE_D, typename LD>
__device__ __forceinline__ void fv_cell(const LD& ld, int i, int j, V dx, V dy,
                                        V g, V delta, V dry_eps, V dt,
                                        int parts, V out[3]) {
  Prim<V> P[5];
  Face<V> Lm, Rm, L0, R0, Lp, Rp;
  V Dm_e[3], Dp_e[3], Dm_w[3], Dp_w[3], I[3];
  Cell<V> c0 = ld(i, j);
  V fx[3] = {V(0), V(0), V(0)}, fy[3] = {V(0), V(0), V(0)};
  if (parts & 1) {
#pragma unroll
    for (int s = 0; s < 5; ++s)
      P[s] = prim(s == 2 ? c0 : ld(i - 2 + s, j), true, delta, ONE_D);
    reconstruct(P[0], P[1], P[2], dry_eps, Lm, Rm);
    reconstruct(P[1], P[2], P[3], dry_eps, L0, R0);
    reconstruct(P[2], P[3], P[4], dry_eps, Lp, Rp);
    pvm(R0, Lp, g, dry_eps, Dm_e, Dp_e);
    pvm(Rm, L0, g, dry_eps, Dm_w, Dp_w);
    interior(L0, R0, c0.h, g, I);
#pragma unroll
    for (int m = 0; m < 3; ++m) fx[m] = (Dm_e[m] + Dp_w[m]) + I[m];
  }
  if (!ONE_D && (parts & 2)) {
#pragma unroll
    for (int s = 0; s < 5; ++s)
      P[s] = prim(s == 2 ? c0 : ld(i, j - 2 + s), false, delta, false);
    reconstruct(P[0], P[1], P[2], dry_eps, Lm, Rm);
    reconstruct(P[1], P[2], P[3], dry_eps, L0, R0);
    reconstruct(P[2], P[3], P[4], dry_eps, Lp, Rp);
    pvm(R0, Lp, g, dry_eps, Dm_e, Dp_e);
    pvm(Rm, L0, g, dry_eps, Dm_w, Dp_w);
    interior(L0, R0, c0.h, g, I);
#pragma unroll
    for (int m = 0; m < 3; ++m) fy[m] = (Dm_e[m] + Dp_w[m]) + I[m];
  }
  // out[0] is the stored depth value (h, or eta in FP32: the same update)
  if (ONE_D) {
    out[0] = c0.s - dt * (fx[0] / dx);
    out[1] = c0.q1 - dt * (fx[1] / dx);
    out[2] = V(0);
  } else {
    out[0] = c0.s - dt * (fx[0] / dx + fy[0] / dy);
    out[1] = c0.q1 - dt * (fx[1] / dx + fy[2] / dy);
    out[2] = c0.q2 - dt * (fx[2] / dx + fy[1] / dy);
  }
}

// positivity clamp (mass added counted), dry cells without discharge, and
// the Manning friction
// discretised semi-implicitly (q implicit, |u| and h explicit) on the stage's
// finite-volume result: q <- q / (1 + dt g n^2 |u| / h^(4/3)), |u| from the
// desingularised velocities (Section 4.5)
// ss: the stored depth value of the stage result (h, or eta in FP32), Hc the
// cell's still-water depth
template <typename T>
__device__ __forceinline__ void fv_finish(T& ss, T Hc, T& qa, T& qb,
                                          T dry_eps, double dx, double dy,
                                          double& clamp, T fric, T dt,
                                          T delta) {
  T hs = Store<T>::depth(ss, Hc);
  if (hs < T(0)) {
    clamp = -(double)hs * dx * dy;
    hs = T(0);
    ss = Store<T>::of_depth(T(0), Hc);
  }
  if (hs <= dry_eps) {
    qa = T(0);
    qb = T(0);
  } else if (fric > T(0)) {
    const T u = desing(hs, qa, delta), v = desing(hs, qb, delta);
    const T den = T(1) + dt * fric * sqrt(u * u + v * v) / (hs * cbrt(hs));
    qa = qa / den;
    qb = qb / den;
  }
}

// The 2D stage on a tile of kFvTX x kFvTY cells: the primitive values of the
// tile and of a halo of 2 cells are formed once into LDS (the loads of the
// halo and of the thread's own cell issued first); each thread then
// evaluates the east and north edges of its cell (the tile's first column
// and row also get their west and south edges), and every edge's
// fluctuations go to both of its cells.  Each cell sums them with its volume
// terms exactly as fv_cell does, so the result is the same to the bit, with
// one evaluation of each edge and of each cell's primitive values instead of
// two and five.
template <typename T>
__device__ __forceinline__ void fv_tile_body(const FvArgs<T>& a, int bid) {
  constexpr int TX = kFvTX, TY = kFvTY, RX = TX + 4, RY = TY + 4;
  __shared__ T ph[RY * RX], pu[RY * RX], pv[RY * RX], pe[RY * RX];
  // FP32 bulk: stored depth values and reference levels (limiter's depth
  // differences, dh_of)
  constexpr bool kS = Store<T>::kEta;
  __shared__ T pS[kS ? RY * RX : 1], pR[kS ? RY * RX : 1];
  // fluctuations of x-edge e of a tile row (e: west edge of column e) and of
  // y-edge e of a tile column; m = to the cell below e, p = to the one above
  constexpr int NXE = (TX + 1) * TY, NYE = TX * (TY + 1);
  __shared__ T xm[3 * NXE], xp[3 * NXE];
  __shared__ T ym[3 * NYE], yp[3 * NYE];
  const int nx = a.nx, ny = a.ny;
  const int txs = a.tiles_x();
  const int i0 = (bid % txs) * TX, j0 = (bid / txs) * TY;
  const T g = a.g, delta = a.delta, dry_eps = a.dry_eps;
  const int tid = (int)threadIdx.x;
  const int tx = tid % TX, ty = tid / TX;
  const int cx = tx + 2, cy = ty + 2;  // the thread's cell in the region
  const int i = i0 + tx, j = j0 + ty;
  const bool own = i < nx && j < ny;
  const int n = j * nx + i;
  // the thread's own inputs, in flight while the tile is formed
  T q10 = T(0), q20 = T(0), s0 = T(0), Hc = T(0);
  if (own) {
    q10 = a.q1[n];
    q20 = a.q2[n];
    if constexpr (kS) s0 = a.h[n];
    Hc = a.H[n];
  }
  const T dt = (T)(*a.dtp);
  constexpr int NRG = (RX * RY + kBlock - 1) / kBlock;
  Cell<T> cl[NRG];
#pragma unroll
  for (int u = 0; u < NRG; ++u) {  // every load of the tile issued first
    const int r = tid + u * kBlock;
    const int ii = i0 - 2 + r % RX, jj = j0 - 2 + r / RX;
    // the cells a grid cell's stencil reads
    if (r < RX * RY && ii <= nx + 1 && jj <= ny + 1)
      cl[u] = load_cell(a.h, a.q1, a.q2, a.H, ii, jj, nx, ny, false, a.open);
  }
#pragma unroll
  for (int u = 0; u < NRG; ++u) {
    const int r = tid + u * kBlock;
    if (r >= RX * RY) break;
    const int ii = i0 - 2 + r % RX, jj = j0 - 2 + r / RX;
    T h = T(0), uu = T(0), vv = T(0), e = T(0), sv = T(0), Rv = T(0);
    if (ii <= nx + 1 && jj <= ny + 1) {
      const Cell<T>& c = cl[u];
      h = c.h;
      uu = desing(c.h, c.q1, delta);
      vv = desing(c.h, c.q2, delta);
      e = c.eta;
      if constexpr (kS) {
        sv = c.s;
        Rv = Store<T>::ref(c.H);
      }
    }
    ph[r] = h;
    pu[r] = uu;
    pv[r] = vv;
    pe[r] = e;
    if constexpr (kS) {
      pS[r] = sv;
      pR[r] = Rv;
    }
  }
  __syncthreads();
  // primitive values at region place q with the normal velocity from un
  // and the tangential one from ut
  auto prim_at = [&](int q, const T* un, const T* ut) {
    Prim<T> p;
    p.h = ph[q];
    p.un = un[q];
    p.ut = ut[q];
    p.eta = pe[q];
    if constexpr (kS) {
      p.s = pS[q];
      p.R = pR[q];
    } else {
      p.s = p.h;
      p.R = T(0);
    }
    return p;
  };
  // edge between region columns c and c + 1 of region row r (x), kept at
  // index e of tile row r - 2; between region rows r and r + 1 of region
  // column c (y), kept at index e of tile column c - 2
  auto x_edge = [&](int c, int r, int e) {
    Face<T> La, Ra, Lb, Rb;
    const int q = r * RX + c;
    reconstruct(prim_at(q - 1, pu, pv), prim_at(q, pu, pv),
                prim_at(q + 1, pu, pv), dry_eps, La, Ra);
    reconstruct(prim_at(q, pu, pv), prim_at(q + 1, pu, pv),
                prim_at(q + 2, pu, pv), dry_eps, Lb, Rb);
    T Dm[3], Dp[3];
    pvm(Ra, Lb, g, dry_eps, Dm, Dp);
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      xm[m * NXE + (r - 2) * (TX + 1) + e] = Dm[m];
      xp[m * NXE + (r - 2) * (TX + 1) + e] = Dp[m];
    }
  };
  auto y_edge = [&](int c, int r, int e) {
    Face<T> La, Ra, Lb, Rb;
    const int q = r * RX + c;
    reconstruct(prim_at(q - RX, pv, pu), prim_at(q, pv, pu),
                prim_at(q + RX, pv, pu), dry_eps, La, Ra);
    reconstruct(prim_at(q, pv, pu), prim_at(q + RX, pv, pu),
                prim_at(q + 2 * RX, pv, pu), dry_eps, Lb, Rb);
    T Dm[3], Dp[3];
    pvm(Ra, Lb, g, dry_eps, Dm, Dp);
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      ym[m * NYE + e * TX + (c - 2)] = Dm[m];
      yp[m * NYE + e * TX + (c - 2)] = Dp[m];
    }
  };
  x_edge(cx, cy, tx + 1);  // east edge
  y_edge(cx, cy, ty + 1);  // north edge
  if (tid < TY)            // west edges of the tile's rows
    x_edge(1, tid + 2, 0);
  else if (tid >= 64 && tid < 64 + TX)
    y_edge(tid - 64 + 2, 1, 0);  // south edges of its columns
  // the cell's own reconstructions for its volume terms
  Face<T> Lx, Rx, Ly, Ry;
  {
    const int q = cy * RX + cx;
    reconstruct(prim_at(q - 1, pu, pv), prim_at(q, pu, pv),
                prim_at(q + 1, pu, pv), dry_eps, Lx, Rx);
    reconstruct(prim_at(q - RX, pv, pu), prim_at(q, pv, pu),
                prim_at(q + RX, pv, pu), dry_eps, Ly, Ry);
  }
  __syncthreads();
  double clamp_local = 0.0;
  if (own) {
    const T h0 = ph[cy * RX + cx];
    // the stored value of the cell (FP64: h0 itself)
    if constexpr (!kS) s0 = h0;
    T Ix[3], Iy[3], fx[3], fy[3];
    interior(Lx, Rx, h0, g, Ix);
    interior(Ly, Ry, h0, g, Iy);
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      fx[m] = (xm[m * NXE + ty * (TX + 1) + tx + 1] +
               xp[m * NXE + ty * (TX + 1) + tx]) +
              Ix[m];
      fy[m] = (ym[m * NYE + (ty + 1) * TX + tx] + yp[m * NYE + ty * TX + tx]) +
              Iy[m];
    }
    T hs = s0 - dt * (fx[0] / a.dx + fy[0] / a.dy);
    T qa = q10 - dt * (fx[1] / a.dx + fy[2] / a.dy);
    T qb = q20 - dt * (fx[2] / a.dx + fy[1] / a.dy);
    fv_finish(hs, Hc, qa, qb, dry_eps, (double)a.dx, (double)a.dy,
              clamp_local, a.fric, dt, a.delta);
    a.oh[n] = hs;
    a.oq1[n] = qa;
    a.oq2[n] = qb;
  }
  double s = block_sum(clamp_local);
  if (threadIdx.x == 0 && s > 0.0) atomicAdd(a.clamped, s);
}

template <typename T, bool ONE_D>
__device__ __forceinline__ void fv_body(const FvArgs<T>& a, int bid) {
  if constexpr (!ONE_D) {
    fv_tile_body<T>(a, bid);
  } else {
    const int n = bid * kBlock + (int)threadIdx.x;
    double clamp_local = 0.0;
    if (n < a.nx) {
      T dt = (T)(*a.dtp);
      CellLoader<T, true> ld{a.h, a.q1, a.q2, a.H, a.nx, 1, a.open};
      T out[3];
      fv_cell<T, true>(ld, n, 0, a.dx, a.dy, a.g, a.delta, a.dry_eps, dt, 3,
                       out);
      T hs = out[0], qa = out[1], qb = out[2];
      fv_finish(hs, a.H[n], qa, qb, a.dry_eps, (double)a.dx, 1.0, clamp_local,
                a.fric, dt, a.delta);
      a.oh[n] = hs;
      a.oq1[n] = qa;
    }
    double s = block_sum(clamp_local);
    if (threadIdx.x == 0 && s > 0.0) atomicAdd(a.clamped, s);
  }
}

// -------------------------------------------------------------------------
// breaking terms (Section 3): nu = max(0, 1 - div q / U1) h |div q|,
// U1 = B1 sqrt(g h); q += dt 2 nu (div u) grad H; rw = 2 nu div u at cells.
// -------------------------------------------------------------------------
template <typename T>
struct BreakCellsArgs {
  int nx, ny;
  T dx, dy, g, delta, dry_eps, b1;
  const T *h, *q1, *q2, *H;
  const double* dtp;
  T *oq1, *oq2, *rw;
  int open;  // open sides (kOpen*)
  __host__ __device__ int nblocks() const { return (nx * ny + kBlock - 1) / kBlock; }
};

template <typename T, bool ONE_D>
__device__ __forceinline__ void break_cells_body(const BreakCellsArgs<T>& a,
                                                 int bid) {
  const int n = bid * kBlock + (int)threadIdx.x;
  const int nx = a.nx, ny = a.ny;
  const T dx = a.dx, dy = a.dy, g = a.g, delta = a.delta, dry_eps = a.dry_eps,
          b1 = a.b1;
  const T* __restrict__ h = a.h;
  const T* __restrict__ q1 = a.q1;
  const T* __restrict__ q2 = a.q2;
  const T* __restrict__ H = a.H;
  if (n >= nx * ny) return;
  int i = n % nx, j = n / nx;
  T dt = (T)(*a.dtp);
  Cell<T> e = load_cell(h, q1, q2, H, i + 1, j, nx, ny, ONE_D, a.open);
  Cell<T> w = load_cell(h, q1, q2, H, i - 1, j, nx, ny, ONE_D, a.open);
  T divq = (e.q1 - w.q1) / (T(2) * dx);
  T divu = (desing(e.h, e.q1, delta) - desing(w.h, w.q1, delta)) / (T(2) * dx);
  T Hx = (e.H - w.H) / (T(2) * dx);
  T Hy = T(0);
  if (!ONE_D) {
    Cell<T> nn = load_cell(h, q1, q2, H, i, j + 1, nx, ny, false, a.open);
    Cell<T> ss = load_cell(h, q1, q2, H, i, j - 1, nx, ny, false, a.open);
    divq += (nn.q2 - ss.q2) / (T(2) * dy);
    divu += (desing(nn.h, nn.q2, delta) - desing(ss.h, ss.q2, delta)) /
            (T(2) * dy);
    Hy = (nn.H - ss.H) / (T(2) * dy);
  }
  T hc = Store<T>::depth(h[n], H[n]);
  T nu = T(0);
  if (hc > dry_eps) {
    T U1 = b1 * sqrt(g * hc);
    T B = T(1) - divq / U1;
    if (B > T(0)) nu = B * hc * fabs(divq);
  }
  T r = T(2) * nu * divu;
  a.rw[n] = r;
  a.oq1[n] = q1[n] + dt * r * Hx;
  if (!ONE_D) a.oq2[n] = q2[n] + dt * r * Hy;
}

template <typename T>
struct BreakCornersArgs {
  int nx, ny;
  T delta;
  const T *h, *rw, *H;
  const double* dtp;
  const T* w_in;
  T* w_out;
  int open;  // boundary mask (kOpen*, kPer*)
  __host__ __device__ int nblocks(bool one_d) const {
    return ((nx + 1) * (one_d ? 1 : ny + 1) + kBlock - 1) / kBlock;
  }
};

template <typename T, bool ONE_D>
__device__ __forceinline__ void break_corners_body(
    const BreakCornersArgs<T>& a, int bid) {
  const int nx = a.nx, ny = a.ny;
  const T delta = a.delta;
  const T* __restrict__ h = a.h;
  const T* __restrict__ rw = a.rw;
  const T* __restrict__ H = a.H;
  int ncx = nx + 1, ncy = ONE_D ? 1 : ny + 1;
  auto dep = [&](int m) { return Store<T>::depth(h[m], H[m]); };
  const int n = bid * kBlock + (int)threadIdx.x;
  if (n >= ncx * ncy) return;
  int k = n % ncx, l = n / ncx;
  T dt = (T)(*a.dtp);
  T hc, rwc;
  // the cells around the corner: mirrored at a wall (an open end's first
  // ghost is the same cell), wrapped on a periodic line
  const bool px = a.open & kPerX, py = a.open & kPerY;
  if (ONE_D) {
    int W = ghost_src(k - 1, nx, false, false, px);
    int E = ghost_src(k, nx, false, false, px);
    hc = T(0.5) * (dep(W) + dep(E));
    rwc = T(0.5) * (rw[W] + rw[E]);
  } else {
    int im = ghost_src(k - 1, nx, false, false, px);
    int ip = ghost_src(k, nx, false, false, px);
    int jm = ghost_src(l - 1, ny, false, false, py);
    int jp = ghost_src(l, ny, false, false, py);
    int SW = jm * nx + im, SE = jm * nx + ip, NW = jp * nx + im,
        NE = jp * nx + ip;
    hc = T(0.25) * (dep(SW) + dep(SE) + dep(NW) + dep(NE));
    rwc = T(0.25) * (rw[SW] + rw[SE] + rw[NW] + rw[NE]);
  }
  a.w_out[n] = a.w_in[n] + dt * desing(hc, rwc, delta);
}

// -------------------------------------------------------------------------
// Energy-consistent vertical momentum (the form named after eq. 7):
// (hw)_t + div(hw u) = p, i.e. h (w_t + u . grad w) = p, so each stage's
// hyperbolic step also carries w with the flow before the pressure step.
// First-order upwind at corner (k, l) with the desingularised velocity of
// the means of h and q over the cells around the corner (stage input V):
//   w* = w - dt [u (w - w_W)/dx or u (w_E - w)/dx, by the sign of u,
//                + the same along y];
// corners past a wall or an open side reflect as the pressure's do, wrap on
// a periodic line; a dry corner keeps its w.
// -------------------------------------------------------------------------
template <typename T>
struct AdvectWArgs {
  int nx, ny;
  T dx, dy, delta, dry_eps;
  const T *h, *q1, *q2, *H;  // stage input V
  const T* w_in;
  const double* dtp;
  T* w_out;
  int open;  // boundary mask (kOpen*, kPer*)
  __host__ __device__ int nblocks(bool one_d) const {
    return ((nx + 1) * (one_d ? 1 : ny + 1) + kBlock - 1) / kBlock;
  }
};

// the stored corner that corner k of a line of n cells reads: reflected
// about the end corner (walls, open ends), wrapped on a periodic line
__device__ __forceinline__ int corner_src(int k, int n, bool per) {
  if (per) return wrap_corner(k, n);
  return k < 0 ? -k : (k > n ? 2 * n - k : k);
}

template <typename T, bool ONE_D>
__global__ void __launch_bounds__(kBlock) k_advect_w(AdvectWArgs<T> a) {
  const int nx = a.nx, ny = a.ny;
  const int ncx = nx + 1, ncy = ONE_D ? 1 : ny + 1;
  const int n = xcd_bid() * kBlock + (int)threadIdx.x;
  if (n >= ncx * ncy) return;
  const int k = n % ncx, l = n / ncx;
  CellLoader<T, ONE_D> ld{a.h, a.q1, a.q2, a.H, nx, ONE_D ? 1 : ny, a.open};
  T hc, qc1, qc2 = T(0);
  if (ONE_D) {
    const Cell<T> W = ld(k - 1, 0), E = ld(k, 0);
    hc = T(0.5) * (W.h + E.h);
    qc1 = T(0.5) * (W.q1 + E.q1);
  } else {
    const Cell<T> SW = ld(k - 1, l - 1), SE = ld(k, l - 1), NW = ld(k - 1, l),
                  NE = ld(k, l);
    hc = T(0.25) * (SW.h + SE.h + NW.h + NE.h);
    qc1 = T(0.25) * (SW.q1 + SE.q1 + NW.q1 + NE.q1);
    qc2 = T(0.25) * (SW.q2 + SE.q2 + NW.q2 + NE.q2);
  }
  const T w = a.w_in[n];
  if (hc <= a.dry_eps) {
    a.w_out[n] = w;
    return;
  }
  const bool px = a.open & kPerX, py = a.open & kPerY;
  auto wat = [&](int kk, int ll) {
    return a.w_in[corner_src(ll, ny, py) * ncx + corner_src(kk, nx, px)];
  };
  const T dt = (T)(*a.dtp);
  const T u = desing(hc, qc1, a.delta);
  const T ddx = u > T(0) ? (w - wat(k - 1, ONE_D ? 0 : l)) / a.dx
                         : (wat(k + 1, ONE_D ? 0 : l) - w) / a.dx;
  T adv = u * ddx;
  if (!ONE_D) {
    const T v = desing(hc, qc2, a.delta);
    const T ddy = v > T(0) ? (w - wat(k, l - 1)) / a.dy
                           : (wat(k, l + 1) - w) / a.dy;
    adv = adv + v * ddy;
  }
  a.w_out[n] = w - dt * adv;
}

// -------------------------------------------------------------------------
// pressure system, 2D: closed-form 5-point coefficients at every corner.
// zeta = h - 2H, X = (zeta_{i+1} - zeta_{i-1})/2, Y alike; pair averages
// over the east/west/north/south cells of the corner; walls folded.
// -------------------------------------------------------------------------
template <typename T>
struct AssembleArgs {
  int nx, ny;
  T dx, dy;
  const T *h, *q1, *q2, *H, *w;
  const double* dtp;
  T *diag, *cE, *cW, *cN, *cS, *rhs;
  int open;  // open sides (kOpen*)
  unsigned* nondom;  // count of rows not strictly dominant (or null)
  // one workgroup per tile of kAsmTX x kAsmTY corners
  __host__ __device__ int nblocks() const;
};
constexpr int kAsmTX = 32, kAsmTY = 8;
static_assert(kAsmTX * kAsmTY == kBlock, "one thread per tile corner");
template <typename T>
__host__ __device__ int AssembleArgs<T>::nblocks() const {
  return ((nx + 1 + kAsmTX - 1) / kAsmTX) * ((ny + 1 + kAsmTY - 1) / kAsmTY);
}

// the Gershgorin check of Section 5 on one assembled row, in FP64 with the
// absolute values summed E, W, N, S
template <typename T>
__device__ __forceinline__ void count_nondominant(unsigned* cnt, T d, T e,
                                                  T w, T n, T s) {
  if (!cnt) return;
  const double off = fabs((double)e) + fabs((double)w) + fabs((double)n) +
                     fabs((double)s);
  if (!((double)d > off)) atomicAdd(cnt, 1u);
}

// The five-point row and right-hand side at corner (k, l) from the mirrored
// cells of `ld`; wc = w* at the corner.  Out: diag, cE, cW, cN, cS, rhs.
template <typename V, typename LD>
__device__ __forceinline__ void assemble_row(const LD& ld, int k, int l, int nx,
                                             int ny, V dx, V dy, V wc, V dt,
                                             V row[6], int bc = 0) {
  const int ci[4] = {k - 1, k, k - 1, k};  // SW, SE, NW, NE
  const int cj[4] = {l - 1, l - 1, l, l};
  V hh[4], zz[4], XX[4], YY[4], a1[4], a2[4];  // a1, a2: q1, q2 of the cells
  auto zeta = [&](int i, int j) { return zeta_of(ld(i, j)); };
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    Cell<V> c = ld(ci[s], cj[s]);
    hh[s] = c.h;
    a1[s] = c.q1;
    a2[s] = c.q2;
    zz[s] = zeta_of(c);
    XX[s] = (zeta(ci[s] + 1, cj[s]) - zeta(ci[s] - 1, cj[s])) / V(2);
    YY[s] = (zeta(ci[s], cj[s] + 1) - zeta(ci[s], cj[s] - 1)) / V(2);
  }
  const int SW = 0, SE = 1, NW = 2, NE = 3;
  V hc = V(0.25) * (hh[SW] + hh[SE] + hh[NW] + hh[NE]);
  V hE = V(0.5) * (hh[SE] + hh[NE]), hW = V(0.5) * (hh[SW] + hh[NW]);
  V hN = V(0.5) * (hh[NW] + hh[NE]), hS = V(0.5) * (hh[SW] + hh[SE]);
  V XE = V(0.5) * (XX[SE] + XX[NE]), XW = V(0.5) * (XX[SW] + XX[NW]);
  V YN = V(0.5) * (YY[NW] + YY[NE]), YS = V(0.5) * (YY[SW] + YY[SE]);
  V sx = V(0.5) * (zz[SE] + zz[NE]) - V(0.5) * (zz[SW] + zz[NW]);
  V sy = V(0.5) * (zz[NW] + zz[NE]) - V(0.5) * (zz[SW] + zz[SE]);
  V q1E = V(0.5) * (a1[SE] + a1[NE]), q1W = V(0.5) * (a1[SW] + a1[NW]);
  V q2N = V(0.5) * (a2[NW] + a2[NE]), q2S = V(0.5) * (a2[SW] + a2[SE]);
  V dx2 = dx * dx, dy2 = dy * dy;
  V d = V(16) +
        ((V(2) * hc + sx) * (XW + V(2) * hW) -
         (V(2) * hc - sx) * (XE - V(2) * hE)) / dx2 +
        ((V(2) * hc + sy) * (YS + V(2) * hS) -
         (V(2) * hc - sy) * (YN - V(2) * hN)) / dy2;
  V e = -(V(2) * hc - sx) * (XE + V(2) * hE) / dx2;
  V wv = (V(2) * hc + sx) * (XW - V(2) * hW) / dx2;
  V nn = -(V(2) * hc - sy) * (YN + V(2) * hN) / dy2;
  V ss = (V(2) * hc + sy) * (YS - V(2) * hS) / dy2;
  V Bs = ((V(2) * hc - sx) * q1E - (V(2) * hc + sx) * q1W) / dx +
         ((V(2) * hc - sy) * q2N - (V(2) * hc + sy) * q2S) / dy +
         V(4) * hc * wc;
  V r = -(V(4) / dt) * Bs;
  // walls fold the mirrored neighbour into the inner one; a periodic line
  // keeps both (its end corners reach across the seam)
  if (!(bc & kPerX)) {
    if (k == 0) { e = e + wv; wv = V(0); }
    if (k == nx) { wv = wv + e; e = V(0); }
  }
  if (!(bc & kPerY)) {
    if (l == 0) { nn = nn + ss; ss = V(0); }
    if (l == ny) { ss = ss + nn; nn = V(0); }
  }
  row[0] = d;
  row[1] = e;
  row[2] = wv;
  row[3] = nn;
  row[4] = ss;
  row[5] = r;
}

// The rows of a tile of kAsmTX x kAsmTY corners: the (mirrored) cells the
// tile's rows read -- those around its corners and their neighbours, a
// block of (TX + 3) x (TY + 3) -- are loaded once into LDS, and every corner
// forms its row from them with assemble_row, as from the bulk arrays.
template <typename T>
__device__ __forceinline__ void assemble2d_body(const AssembleArgs<T>& a,
                                                int bid) {
  constexpr int TX = kAsmTX, TY = kAsmTY, RX = TX + 3, RY = TY + 3;
  __shared__ T ch[RY * RX], cq1[RY * RX], cq2[RY * RX], cs[RY * RX],
      cH[RY * RX];
  const int nx = a.nx, ny = a.ny;
  const int ncx = nx + 1, ncy = ny + 1;
  const int tpx = (ncx + TX - 1) / TX;
  const int k0 = (bid % tpx) * TX, l0 = (bid / tpx) * TY;
  const int tid = (int)threadIdx.x;
  const int k = k0 + tid % TX, l = l0 + tid / TX;
  const bool own = k < ncx && l < ncy;
  const int n = l * ncx + k;
  const T wc = own ? a.w[n] : T(0);
  const T dt = (T)(*a.dtp);
  for (int r = tid; r < RX * RY; r += kBlock) {
    const int i = k0 - 2 + r % RX, j = l0 - 2 + r / RX;
    Cell<T> c{T(0), T(0), T(0), T(0), T(0), T(0)};
    if (i <= nx + 1 && j <= ny + 1)  // the cells a row reads
      c = load_cell(a.h, a.q1, a.q2, a.H, i, j, nx, ny, false, a.open);
    ch[r] = c.h;
    cq1[r] = c.q1;
    cq2[r] = c.q2;
    cs[r] = c.s;
    cH[r] = c.H;
  }
  __syncthreads();
  if (!own) return;
  // the staged cell at grid position (i, j) (eta is not read by the row)
  auto ld = [&](int i, int j) {
    const int r = (j - l0 + 2) * RX + (i - k0 + 2);
    return Cell<T>{ch[r], cq1[r], cq2[r], cH[r], T(0), cs[r]};
  };
  T row[6];
  assemble_row<T>(ld, k, l, nx, ny, a.dx, a.dy, wc, dt, row, a.open);
  a.diag[n] = row[0];
  a.cE[n] = row[1];
  a.cW[n] = row[2];
  a.cN[n] = row[3];
  a.cS[n] = row[4];
  a.rhs[n] = row[5];
  count_nondominant(a.nondom, row[0], row[1], row[2], row[3], row[4]);
}

// 1D: eq. (43) coefficients, rows scaled by dx^2, with the right-hand side
// -(8 dx^2/dt)(h q_x - q (2 eta - h)_x + 2 h w) at the corner.
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_assemble1d(int nx, T dx, const T* __restrict__ h,
                 const T* __restrict__ q, const T* __restrict__ H,
                 const T* __restrict__ w, const double* __restrict__ dtp,
                 T* __restrict__ a, T* __restrict__ b, T* __restrict__ c,
                 T* __restrict__ rhs, int open, unsigned* nondom) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k > nx) return;
  T dt = (T)(*dtp);
  const bool ow = open & kOpenW, oe = open & kOpenE, per = open & kPerX;
  auto zeta = [&](int i) {
    int m = ghost_src(i, nx, ow, oe, per);
    if constexpr (Store<T>::kEta)
      return H[m] > T(0) ? h[m] - H[m] : h[m] - T(2) * H[m];
    else
      return h[m] - T(2) * H[m];
  };
  auto qv = [&](int i) {
    int m = ghost_src(i, nx, ow, oe, per);
    return (m != i && !per && !(i < 0 ? ow : oe)) ? -q[m] : q[m];
  };
  int Wi = ghost_src(k - 1, nx, false, false, per);
  int Ei = ghost_src(k, nx, false, false, per);
  T hW = Store<T>::depth(h[Wi], H[Wi]), hE = Store<T>::depth(h[Ei], H[Ei]);
  T hc = T(0.5) * (hE + hW);
  T zW = zeta(k - 1), zE = zeta(k);
  T xiW = dx * ((zE - zeta(k - 2)) / (T(2) * dx));
  T xiE = dx * ((zeta(k + 1) - zW) / (T(2) * dx));
  T xic = dx * ((zE - zW) / dx);
  T ai = (xiW - T(2) * hW) * (xic + T(2) * hc);
  T bi = T(16) * dx * dx + xic * (xiW + xiE + T(2) * hW - T(2) * hE) +
         T(2) * hc * (xiW - xiE + T(4) * hc);
  T ci = (xiE + T(2) * hE) * (xic - T(2) * hc);
  T qE = qv(k), qW = qv(k - 1);
  T qc = T(0.5) * (qE + qW);
  T qxc = (qE - qW) / dx;
  T zxc = (zE - zW) / dx;
  T Bc = hc * qxc - qc * zxc + T(2) * hc * w[k];
  T r = -(T(8) * dx * dx / dt) * Bc;
  if (!per) {  // walls fold the mirrored neighbour (periodic: the cyclic row)
    if (k == 0) { ci = ci + ai; ai = T(0); }
    if (k == nx) { ai = ai + ci; ci = T(0); }
  }
  a[k] = ai;
  b[k] = bi;
  c[k] = ci;
  rhs[k] = r;
  count_nondominant(nondom, bi, ci, ai, T(0), T(0));
}

// Thomas algorithm (Section 4.3) for the tridiagonal system (42), in FP64 by
// one thread: the 1D channel is small and the elimination is sequential.
template <typename T>
__global__ void k_thomas(int n, const T* __restrict__ a, const T* __restrict__ b,
                         const T* __restrict__ c, const T* __restrict__ d,
                         double* __restrict__ x, double* __restrict__ cp,
                         double* __restrict__ dp, int* __restrict__ flags) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double b0 = (double)b[0];
  if (!(b0 != 0.0)) { atomicOr(flags, 2); return; }
  cp[0] = (double)c[0] / b0;
  dp[0] = (double)d[0] / b0;
  for (int k = 1; k < n; ++k) {
    double m = (double)b[k] - (double)a[k] * cp[k - 1];
    if (!(m != 0.0)) { atomicOr(flags, 2); return; }
    cp[k] = (double)c[k] / m;
    dp[k] = ((double)d[k] - (double)a[k] * dp[k - 1]) / m;
  }
  double xn = dp[n - 1];
  x[n - 1] = xn;
  for (int k = n - 2; k >= 0; --k) {
    xn = dp[k] - cp[k] * xn;
    x[k] = xn;
  }
}

// Periodic 1D channel (Section 4.4, item 1): the n = nx distinct corners form
// a cyclic tridiagonal system (row 0 reaches corner n - 1 through a[0], row
// n - 1 reaches corner 0 through c[n - 1]), solved by the Sherman-Morrison
// modification of the Thomas algorithm: with gamma = -b[0], two tridiagonal
// solves with the diagonal b[0] - gamma, b[1], ..., b[n-1] - c[n-1] a[0] /
// gamma -- of the right-hand side and of u = (gamma, 0, ..., 0, c[n-1]) --
// and the rank-one correction x -= (x0 + a[0] x_{n-1} / gamma) / (1 + z0 +
// a[0] z_{n-1} / gamma) z.  In FP64 by one thread; corner n gets corner 0's
// value.  bb, z, cp, dp: n FP64 work values each.
template <typename T>
__global__ void k_thomas_cyclic(int n, const T* __restrict__ a,
                                const T* __restrict__ b,
                                const T* __restrict__ c,
                                const T* __restrict__ d,
                                double* __restrict__ x,
                                double* __restrict__ bb,
                                double* __restrict__ z,
                                double* __restrict__ cp,
                                double* __restrict__ dp,
                                int* __restrict__ flags) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const double alpha = (double)c[n - 1], beta = (double)a[0];
  const double gamma = -(double)b[0];
  if (!(gamma != 0.0)) { atomicOr(flags, 2); return; }
  for (int k = 0; k < n; ++k) bb[k] = (double)b[k];
  bb[0] = (double)b[0] - gamma;
  bb[n - 1] = (double)b[n - 1] - alpha * beta / gamma;
  // one tridiagonal elimination of the right-hand side r into y
  auto tridiag = [&](auto rhs, double* y) -> bool {
    if (!(bb[0] != 0.0)) return false;
    cp[0] = (double)c[0] / bb[0];
    dp[0] = rhs(0) / bb[0];
    for (int k = 1; k < n; ++k) {
      const double m = bb[k] - (double)a[k] * cp[k - 1];
      if (!(m != 0.0)) return false;
      cp[k] = (double)c[k] / m;
      dp[k] = (rhs(k) - (double)a[k] * dp[k - 1]) / m;
    }
    double yn = dp[n - 1];
    y[n - 1] = yn;
    for (int k = n - 2; k >= 0; --k) {
      yn = dp[k] - cp[k] * yn;
      y[k] = yn;
    }
    return true;
  };
  if (!tridiag([&](int k) { return (double)d[k]; }, x)) {
    atomicOr(flags, 2);
    return;
  }
  if (!tridiag([&](int k) {
        return k == 0 ? gamma : (k == n - 1 ? alpha : 0.0);
      }, z)) {
    atomicOr(flags, 2);
    return;
  }
  const double den = 1.0 + z[0] + beta * z[n - 1] / gamma;
  if (!(den != 0.0)) { atomicOr(flags, 2); return; }
  const double fact = (x[0] + beta * x[n - 1] / gamma) / den;
  for (int k = 0; k < n; ++k) x[k] = x[k] - fact * z[k];
  x[n] = x[0];
}

// -------------------------------------------------------------------------
// relaxed Jacobi sweeps of the 2D pressure system, several per launch.
// Sweep k is
//   r = rhs - (diag p + cE pE + cW pW + cN pN + cS pS),
//   p <- p + omega_k (r / diag)
// in FP64 with an FP64 iterate (coefficients in the bulk type), in the order
// of the plain statement, so that FP64 iterates are reproduced exactly.  A workgroup
// owns a BX x BY tile of corners and loads it with a halo of S corners; the
// iterate ping-pongs in LDS and the coefficients stay in registers.  After t
// sweeps the values are exact on the region shrunk by t, so nsw <= S sweeps in
// one launch give the same iterates as nsw separate sweeps.  Outside the
// domain everything is zero (walls are folded into the boundary rows).
// With check, the first sweep max-reduces |r| over the tile -- the size of a
// plain Jacobi update of the input iterate (eq. 32) -- into part[tile], and
// the input iterate of the tile is copied to psave, so that the host can
// decide on convergence while later launches already run; nsw == 0 only
// measures.
// Tiles are assigned XCD-major: workgroup b runs on XCD b % 8, and each XCD
// gets a contiguous band of tile rows, so the halos and the coefficients of
// its band stay in its own L2 from one launch to the next.
// -------------------------------------------------------------------------
constexpr int kSweepB = 1024;  // threads per workgroup (16 waves)
constexpr int kSweepS = 8;     // sweeps per launch (= halo width)
constexpr int kSweepM = 2;     // region points per thread:
                               // (BX+2S)(BY+2S) <= kSweepB * kSweepM
constexpr int kSweepMBig = 3;  // large grids and ensembles: bigger tiles

// per-grid arguments of the sweep kernel
template <typename T>
struct SweepArgs {
  int ncx, ncy, BX, BY, ntx, ntiles;
  int bc = 0;            // boundary mask (kPer*: halos wrap around)
  const T *diag, *cE, *cW, *cN, *cS, *rhs;
  double* p[3];          // iterate buffers
  const double* omega;   // relaxation schedule
  int nom;
  double* part;          // per-tile convergence measures
  // stop on the relative residual: max |rhs| of the system (null: the
  // plain-update measure of eq. 32)
  const double* rmax = nullptr;
  __host__ __device__ int nblocks() const { return 8 * ((ntiles + 7) / 8); }
};

// the measure of one corner at a check: the size of its plain Jacobi
// update, or (relative residual) of its residual
__device__ __forceinline__ double check_term(bool resid, double r,
                                             double rdiag) {
  return resid ? fabs(r) : fabs(r * rdiag);
}
// the check's measure from the maximum of the corner terms
__device__ __forceinline__ double check_measure(const double* rmax,
                                                double m) {
  if (rmax && *rmax > 0.0) return m / *rmax;
  return m;
}

// max |a| of n values (one workgroup; the order does not matter)
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_absmax(long n, const T* __restrict__ a, double* __restrict__ out) {
  double v = 0.0;
  for (long i = threadIdx.x; i < n; i += kBlock) {
    const double x = fabs((double)a[i]);
    v = x > v ? x : v;
  }
  __shared__ double ws[kBlock / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double x = __shfl_xor(v, o, 64);
    v = x > v ? x : v;
  }
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = ws[0];
    for (int w = 1; w < kBlock / 64; ++w) m = ws[w] > m ? ws[w] : m;
    *out = m;
  }
}

constexpr int kFlagWaitBound = 8;  // solver flags: a wait gave up
constexpr int kPersistOmega = 256;  // schedule factors staged in LDS

__device__ __forceinline__ unsigned long long ld_agent_u64(
    unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent_u64(unsigned long long* p,
                                             unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned ld_agent_u32(unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_agent(const double* p) {
  auto* q = reinterpret_cast<unsigned long long*>(const_cast<double*>(p));
  return __longlong_as_double((long long)ld_agent_u64(q));
}
__device__ __forceinline__ void st_agent(double* p, double v) {
  st_agent_u64(reinterpret_cast<unsigned long long*>(p),
               (unsigned long long)__double_as_longlong(v));
}
// this thread's memory operations have completed (and no memory access is
// moved across by the compiler)
__device__ __forceinline__ void wait_memory() {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}
__device__ __forceinline__ bool gave_up(int* flags) {
  return (__hip_atomic_load(flags, __ATOMIC_RELAXED,
                            __HIP_MEMORY_SCOPE_AGENT) &
          kFlagWaitBound) != 0;
}
// per-launch arguments (common to every grid of a batch)
struct SweepLaunch {
  int iin, iout, isave;  // buffers read, written, saved (check launch)
  int k0, nsw, check;
  // single grid: the launch after a check carries one extra workgroup that
  // reduces the check's per-tile measures (complete at the kernel boundary)
  // into E_host and then releases seq into seq_slot (mapped host memory)
  int reduce;
  double* E_host;
  long long* seq_slot;
  long long seq;
};

// COH: the iterate, the saved iterate and the per-tile measures are read and
// written at device scope (coherent across the XCDs' L2s), for the solve
// that runs its launches' work inside one kernel between grid barriers
template <typename T, int B, int S, int M, bool COH = false>
__device__ __forceinline__ void sweep_body(const SweepArgs<T>& a,
                                           const SweepLaunch& L, int bid,
                                           double* lds) {
  const int ncx = a.ncx, ncy = a.ncy, BX = a.BX, BY = a.BY, ntx = a.ntx;
  const T* __restrict__ dgl = a.diag;
  const T* __restrict__ cE = a.cE;
  const T* __restrict__ cW = a.cW;
  const T* __restrict__ cN = a.cN;
  const T* __restrict__ cS = a.cS;
  const T* __restrict__ rhs = a.rhs;
  const double* __restrict__ pin = a.p[L.iin];
  double* __restrict__ pout = a.p[L.iout];
  double* __restrict__ psave = a.p[L.isave];
  const double* __restrict__ omega = a.omega;
  const int nom = a.nom, k0 = L.k0, nsw = L.nsw, check = L.check;
  const int per = a.nblocks() / 8;
  const int tile = (bid % 8) * per + (bid / 8);
  if (tile >= a.ntiles) return;  // uniform over the workgroup
  const int tx = tile % ntx, ty = tile / ntx;
  const int RW = BX + 2 * S, RH = BY + 2 * S, R = RW * RH;
  const int x0 = tx * BX - S, y0 = ty * BY - S;
  double* P0 = lds;
  double* P1 = lds + R;
  // the update in FP64 (also for FP32 coefficients): A p as diag p plus fused
  // multiply-adds of the E, W, N, S neighbours in that order, a product with
  // the correctly rounded reciprocal of the diagonal, and a fused update --
  // the operation order of the oracle, so that FP64 iterates agree bit for bit
  // outside the domain: diag 1, everything else 0 (the iterate stays 0)
  // the row coefficients stay in registers in their storage type and are
  // widened to FP64 for the update (the same values either way)
  T dg[M], ce[M], cw[M], cn[M], cs[M], cr[M];
  int rx[M], ry[M];
#pragma unroll
  for (int m = 0; m < M; ++m) {
    int idx = (int)threadIdx.x + B * m;
    ce[m] = cw[m] = cn[m] = cs[m] = cr[m] = T(0);
    dg[m] = T(1);
    rx[m] = -1;
    ry[m] = -1;
    if (idx < R) {
      rx[m] = idx % RW;
      ry[m] = idx / RW;
      const int ux = x0 + rx[m], uy = y0 + ry[m];  // unwrapped position
      // a periodic direction takes the halo from across the seam (corner
      // ncx - 1 is corner 0 again)
      const int gx = (a.bc & kPerX) ? wrap_corner(ux, ncx - 1) : ux;
      const int gy = (a.bc & kPerY) ? wrap_corner(uy, ncy - 1) : uy;
      double pv = 0.0;
      if (gx >= 0 && gx < ncx && gy >= 0 && gy < ncy) {
        int g = gy * ncx + gx;
        if constexpr (COH)
          pv = ld_agent(pin + g);
        else
          pv = pin[g];
        if (check && rx[m] >= S && rx[m] < S + BX && ry[m] >= S &&
            ry[m] < S + BY && ux < ncx && uy < ncy) {
          if constexpr (COH)
            st_agent(psave + g, pv);
          else
            psave[g] = pv;
        }
        dg[m] = dgl[g];
        ce[m] = cE[g];
        cw[m] = cW[g];
        cn[m] = cN[g];
        cs[m] = cS[g];
        cr[m] = rhs[g];
      }
      P0[idx] = pv;
    }
  }
  double rdg[M];
#pragma unroll
  for (int m = 0; m < M; ++m) rdg[m] = 1.0 / (double)dg[m];
  __syncthreads();
  double e = 0.0;
  const int iters = nsw > 0 ? nsw : 1;
  for (int t = 0; t < iters; ++t) {
    const double om = omega[(k0 + t) % nom];
    const double* src = (t & 1) ? P1 : P0;
    double* dst = (t & 1) ? P0 : P1;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int x = rx[m], y = ry[m];
      if (x > t && x < RW - 1 - t && y > t && y < RH - 1 - t) {
        const int idx = (int)threadIdx.x + B * m;
        const double pc = src[idx];
        T cd = dg[m], c1 = ce[m], c2 = cw[m], c3 = cn[m], c4 = cs[m],
          c5 = cr[m];
        if constexpr (sizeof(T) == 4 && M >= 3) {
          // opaque to loop-invariant code motion: the widening stays here
          // and the floats, not their FP64 copies, live across the sweeps
          // (with 3 points per thread this keeps the kernel within 64
          // registers, i.e. two 1024-thread workgroups per CU)
          asm volatile("" : "+v"(cd), "+v"(c1), "+v"(c2), "+v"(c3), "+v"(c4),
                       "+v"(c5));
        }
        double Ap = (double)cd * pc;
        Ap = fma((double)c1, src[idx + 1], Ap);
        Ap = fma((double)c2, src[idx - 1], Ap);
        Ap = fma((double)c3, src[idx + RW], Ap);
        Ap = fma((double)c4, src[idx - RW], Ap);
        const double res = (double)c5 - Ap;
        const double rd = res * rdg[m];
        const double pn = fma(om, rd, pc);
        if (t == 0 && check && x >= S && x < S + BX && y >= S && y < S + BY) {
          const double ar = check_term(a.rmax != nullptr, res, rdg[m]);
          e = (ar > e || ar != ar) ? ar : e;
        }
        if (nsw > 0) dst[idx] = pn;
      }
    }
    __syncthreads();
  }
  if (nsw > 0) {
    const double* fin = (nsw & 1) ? P1 : P0;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int x = rx[m], y = ry[m];
      if (x >= S && x < S + BX && y >= S && y < S + BY) {
        int gx = x0 + x, gy = y0 + y;
        if (gx < ncx && gy < ncy) {
          if constexpr (COH)
            st_agent(pout + gy * ncx + gx, fin[(int)threadIdx.x + B * m]);
          else
            pout[gy * ncx + gx] = fin[(int)threadIdx.x + B * m];
        }
      }
    }
  }
  if (check) {
    __shared__ double wmax[B / 64];
    double v = wave_max(e);
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double mx = wmax[0];
      for (int w = 1; w < B / 64; ++w)
        mx = (wmax[w] > mx || wmax[w] != wmax[w]) ? wmax[w] : mx;
      if constexpr (COH)
        st_agent(a.part + tile, mx);
      else
        a.part[tile] = mx;
    }
  }
}

// -------------------------------------------------------------------------
// correction (eq. 26-27 in 1D, eq. 36 in 2D) of the cell discharges and the
// corner update w = w* + dt p / h_c (desingularised division), in one launch
// over max(cells, corners) threads.  With COMBINE (second stage) the new
// state is averaged with U^n (TVD-RK2) and each workgroup writes the CFL
// measure max((|u|+c)/dx + (|v|+c)/dy) of its cells to lampart[block].
// With have_p == 0 (hydrostatic mode) the discharges pass through.
// -------------------------------------------------------------------------
template <typename T>
struct CorrectArgs {
  int nx, ny;
  T dx, dy, g, delta, dry_eps;
  int have_p;
  const T *hs, *q1s, *q2s, *H, *ws;
  const double* p;
  const double* dtp;
  T *oq1, *oq2, *w_out, *h_n, *q1_n, *q2_n;
  double* lampart;
  int* flags;
  // generation/absorption zones (Section 4.4), applied with the RK average:
  // weights of the state and targets in the cells and at the corners (null:
  // no zones)
  const T *rm_c, *rt_h, *rt_q1, *rt_q2, *rm_k, *rt_w;
  int open;  // open sides (kOpen*)
  __host__ __device__ int nblocks(bool one_d) const {
    int nc = nx * ny, nk = (nx + 1) * (one_d ? 1 : ny + 1);
    return ((nc > nk ? nc : nk) + kBlock - 1) / kBlock;
  }
};

// Correction of the discharges of cell (i, j) (eq. 26-27 in 1D, eq. 36 in
// 2D) given its stage discharges qa, qb (in/out); `ld` gives the mirrored
// stage cells (h*, H) and `pl(k, l)` the corner pressures.
template <typename V, bool ONE_D, typename LD, typename PL>
__device__ __forceinline__ void correct_cell(const LD& ld, const PL& pl, int i,
                                             int j, V dx, V dy, V dt, V dry_eps,
                                             V& qa, V& qb) {
  auto zeta = [&](int ii, int jj) { return zeta_of(ld(ii, jj)); };
  V hc = ld(i, j).h;
  V zx = (zeta(i + 1, j) - zeta(i - 1, j)) / (V(2) * dx);
  if (ONE_D) {
    V pR = pl(i + 1, 0), pL = pl(i, 0);
    V Tn = -V(0.5) * (hc * ((pR - pL) / dx) + (V(0.5) * (pR + pL)) * zx);
    qa = qa + dt * Tn;
    qb = V(0);
  } else {
    V zy = (zeta(i, j + 1) - zeta(i, j - 1)) / (V(2) * dy);
    V pSW = pl(i, j), pSE = pl(i + 1, j);
    V pNW = pl(i, j + 1), pNE = pl(i + 1, j + 1);
    V TN = -V(0.5) * hc * (pNE - pNW) / dx -
           V(0.5) * (V(0.5) * (pNE + pNW)) * zx;
    V TS = -V(0.5) * hc * (pSE - pSW) / dx -
           V(0.5) * (V(0.5) * (pSE + pSW)) * zx;
    V TE = -V(0.5) * hc * (pNE - pSE) / dy -
           V(0.5) * (V(0.5) * (pNE + pSE)) * zy;
    V TW = -V(0.5) * hc * (pNW - pSW) / dy -
           V(0.5) * (V(0.5) * (pNW + pSW)) * zy;
    qa = qa + dt * (V(0.5) * (TN + TS));
    qb = qb + dt * (V(0.5) * (TE + TW));
  }
  if (hc <= dry_eps) {
    qa = V(0);
    qb = V(0);
  }
}

// w = w* + dt p / h_c at corner (k, l) with the desingularised division
// (Section 4.5); h_c is the mean of the (mirrored) cells around the corner.
template <typename V, bool ONE_D, typename LD>
__device__ __forceinline__ V correct_corner(const LD& ld, int k, int l, V ws,
                                            V pc, V dt, V delta) {
  V hc;
  if (ONE_D)
    hc = V(0.5) * (ld(k - 1, 0).h + ld(k, 0).h);
  else
    hc = V(0.25) * (ld(k - 1, l - 1).h + ld(k, l - 1).h + ld(k - 1, l).h +
                    ld(k, l).h);
  return ws + dt * desing(hc, pc, delta);
}

// corner pressures of the FP64 iterate, read in the bulk type
template <typename T>
struct PLoader {
  const double* p;
  int ncx;
  __device__ __forceinline__ T operator()(int k, int l) const {
    return (T)p[l * ncx + k];
  }
};

template <typename T, bool ONE_D, bool COMBINE>
__device__ __forceinline__ void correct_body(const CorrectArgs<T>& a,
                                             int bid) {
  const int n = bid * kBlock + (int)threadIdx.x;
  const int nx = a.nx, ny = a.ny, have_p = a.have_p;
  const T dx = a.dx, dy = a.dy, g = a.g, delta = a.delta, dry_eps = a.dry_eps;
  const T* __restrict__ hs = a.hs;
  const T* __restrict__ H = a.H;
  const double* __restrict__ p = a.p;
  const int ncx = nx + 1, ncy = ONE_D ? 1 : ny + 1;
  const T dt = (T)(*a.dtp);
  double lam_local = 0.0;
  CellLoader<T, ONE_D> ld{hs, a.q1s, a.q2s, H, nx, ONE_D ? 1 : ny, a.open};
  PLoader<T> pl{p, ncx};
  if (n < nx * ny) {
    int i = n % nx, j = n / nx;
    T hc = hs[n];
    T qa = a.q1s[n], qb = ONE_D ? T(0) : a.q2s[n];
    if (have_p) correct_cell<T, ONE_D>(ld, pl, i, j, dx, dy, dt, dry_eps, qa, qb);
    if (!COMBINE) {
      a.oq1[n] = qa;
      if (!ONE_D) a.oq2[n] = qb;
    } else {
      T hn = T(0.5) * (a.h_n[n] + hc);
      T an = T(0.5) * (a.q1_n[n] + qa);
      T bn = ONE_D ? T(0) : T(0.5) * (a.q2_n[n] + qb);
      if (a.rm_c) {  // U <- m U + (1 - m) U* in the zones
        const T m = a.rm_c[n];
        hn = m * hn + (T(1) - m) * a.rt_h[n];
        an = m * an + (T(1) - m) * a.rt_q1[n];
        if (!ONE_D) bn = m * bn + (T(1) - m) * a.rt_q2[n];
      }
      a.h_n[n] = hn;
      a.q1_n[n] = an;
      if (!ONE_D) a.q2_n[n] = bn;
      if (!isfinite((double)hn) || !isfinite((double)an) ||
          !isfinite((double)bn))
        atomicOr(a.flags, 1);
      const T hd = Store<T>::depth(hn, H[n]);  // hn: the stored value
      if (hd > dry_eps) {
        T cel = sqrt(g * hd);
        T u = desing(hd, an, delta);
        T l = (fabs(u) + cel) / dx;
        if (!ONE_D) {
          T v = desing(hd, bn, delta);
          l = l + (fabs(v) + cel) / dy;
        }
        lam_local = (double)l;
      }
    }
  }
  if (n < ncx * ncy) {
    int k = n % ncx, l = n / ncx;
    T wv = a.ws[n];
    if (have_p)
      wv = correct_corner<T, ONE_D>(ld, k, l, wv, (T)p[n], dt, delta);
    if (COMBINE) {
      T wn = T(0.5) * (a.w_out[n] + wv);
      if (a.rm_k) {
        const T m = a.rm_k[n];
        wn = m * wn + (T(1) - m) * a.rt_w[n];
      }
      a.w_out[n] = wn;
    } else {
      a.w_out[n] = wv;
    }
  }
  if (COMBINE) {
    __shared__ double wmax[kBlock / 64];
    double v = wave_max(lam_local);
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double m = wmax[0];
      for (int w = 1; w < kBlock / 64; ++w)
        m = (wmax[w] > m || wmax[w] != wmax[w]) ? wmax[w] : m;
      a.lampart[bid] = m;
    }
  }
}

// p <- m p + (1 - m) p* at the corners of the zones, after the step's
// correction (other threads of the correction still read p)
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_relax_p(int n, double* __restrict__ p, const T* __restrict__ m,
              const double* __restrict__ pt) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= n) return;
  const double w = (double)m[c];
  p[c] = w * p[c] + (1.0 - w) * pt[c];
}

// CFL measure of a state (used at set_state): per-block maxima of
// (|u|+c)/dx + (|v|+c)/dy over the wet cells into lampart[block]
template <typename T>
struct LambdaArgs {
  int nx, ny;
  T dx, dy, g, delta, dry_eps;
  const T *h, *q1, *q2, *H;
  double* lampart;
  __host__ __device__ int nblocks() const { return (nx * ny + kBlock - 1) / kBlock; }
};

template <typename T, bool ONE_D>
__device__ __forceinline__ void lambda_body(const LambdaArgs<T>& a, int bid) {
  const int n = bid * kBlock + (int)threadIdx.x;
  double lam_local = 0.0;
  if (n < a.nx * a.ny) {
    T hn = Store<T>::depth(a.h[n], a.H[n]);
    if (hn > a.dry_eps) {
      T cel = sqrt(a.g * hn);
      T u = desing(hn, a.q1[n], a.delta);
      T l = (fabs(u) + cel) / a.dx;
      if (!ONE_D) {
        T v = desing(hn, a.q2[n], a.delta);
        l = l + (fabs(v) + cel) / a.dy;
      }
      lam_local = (double)l;
    }
  }
  __shared__ double wmax[kBlock / 64];
  double v = wave_max(lam_local);
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = wmax[0];
    for (int w = 1; w < kBlock / 64; ++w)
      m = (wmax[w] > m || wmax[w] != wmax[w]) ? wmax[w] : m;
    a.lampart[bid] = m;
  }
}

// statistics kept on the device between synchronisations
struct DevStats {
  double t;        // simulated time
  double dt_last;  // dt of the last step
  long long step;  // steps since the state was set
  // solves done in one launch each (k_solve_persist), whose sweep counts the
  // host does not see
  long long sweeps_total, solves_total, noconv;
  double measure;  // measure at the end of the last such solve
  int sweeps[2];   // sweeps of the last such solve of each stage
  long long prof_sweeps;  // sweeps of the such solves the host timed
  double depth_sum;       // sum of the depths at the last status read
  // rows of the pressure systems that are not strictly diagonally dominant
  // (Section 5: reported, not enforced): counted by the running step's
  // assemblies, moved to nondom_last at its end
  unsigned nondom_run;
  long long nondom_last;
};


// End of a step (one workgroup): account the step's dt, reduce the per-block
// CFL measures of the new state and set dt = CFL / lambda_max for the next
// step (unless dt is fixed).  Stays on the device.
struct FinalizeArgs {
  double cfl;
  int fixed;
  const double* lampart;
  int nparts;
  double* dt;
  int* flags;
  DevStats* st;
};

__device__ __forceinline__ void finalize_body(const FinalizeArgs& a) {
  double v = 0.0;
  for (int i = threadIdx.x; i < a.nparts; i += blockDim.x) {
    double x = a.lampart[i];
    v = (x > v || x != x) ? x : v;
  }
  __shared__ double wmax[kBlock / 64];
  v = wave_max(v);
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x != 0) return;
  double l = wmax[0];
  for (int w = 1; w < kBlock / 64; ++w)
    l = (wmax[w] > l || wmax[w] != wmax[w]) ? wmax[w] : l;
  if (a.st) {
    double used = *a.dt;
    a.st->t += used;
    a.st->dt_last = used;
    a.st->step += 1;
    a.st->nondom_last = a.st->nondom_run;
    a.st->nondom_run = 0u;
  }
  if (!a.fixed) {
    if (l > 0.0 && isfinite(l)) {
      *a.dt = a.cfl / l;
    } else {
      *a.dt = 0.0;
      atomicOr(a.flags, 4);
    }
  }
}

// max of the per-tile convergence measures of each grid, written to mapped
// host memory, then the check's sequence number (release at system scope)
__global__ void __launch_bounds__(kBlock)
    k_reduce_measure(const double* const* __restrict__ parts,
                     const int* __restrict__ nparts, int ngrids,
                     double* __restrict__ E, long long* seq_slot,
                     long long seq, const double* rmax = nullptr) {
  __shared__ double wmax[kBlock / 64];
  for (int gi = 0; gi < ngrids; ++gi) {
    const double* part = parts[gi];
    double v = 0.0;
    for (int i = threadIdx.x; i < nparts[gi]; i += blockDim.x) {
      double x = part[i];
      v = (x > v || x != x) ? x : v;
    }
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double m = wmax[0];
      for (int w = 1; w < kBlock / 64; ++w)
        m = (wmax[w] > m || wmax[w] != wmax[w]) ? wmax[w] : m;
      E[gi] = check_measure(rmax, m);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    __threadfence_system();
    __hip_atomic_store(seq_slot, seq, __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

__global__ void k_zero_u64(unsigned long long* a) { *a = 0ull; }

template <typename T>
__global__ void k_fill(long n, T v, T* __restrict__ a) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// check of an array handed in as device memory: a non-finite element sets
// bit nf of *flags, a negative one (when neg != 0) bit neg; one atomic per
// workgroup
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_check_values(long n, const T* __restrict__ a, int nf, int neg,
                   int* __restrict__ flags, const T* __restrict__ H = nullptr) {
  const long i = (long)blockIdx.x * kBlock + threadIdx.x;
  int bad_nf = 0, bad_neg = 0;
  if (i < n) {
    // with H: a holds stored depth values, checked as depths
    const double v = H ? (double)Store<T>::depth(a[i], H[i]) : (double)a[i];
    bad_nf = !isfinite(v);
    bad_neg = neg != 0 && v < 0.0;
  }
  bad_nf = __syncthreads_or(bad_nf);
  bad_neg = __syncthreads_or(bad_neg);
  if (threadIdx.x == 0 && (bad_nf || bad_neg))
    atomicOr(flags, (bad_nf ? nf : 0) | (bad_neg ? neg : 0));
}

template <typename Tdst, typename Tsrc>
__global__ void k_convert(int n, const Tsrc* __restrict__ s,
                          Tdst* __restrict__ d) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = (Tdst)s[i];
}

// per-workgroup sums of the depth (in FP64, a fixed tree per workgroup) for
// the water volume
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_depth_sums(long n, const T* __restrict__ h, const T* __restrict__ H,
                 double* __restrict__ part) {
  const long i = (long)blockIdx.x * kBlock + threadIdx.x;
  double v = i < n ? (double)Store<T>::depth(h[i], H[i]) : 0.0;
  __shared__ double ws[kBlock / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) s += ws[w];
    part[blockIdx.x] = s;
  }
}

// the sum of the per-workgroup sums (one workgroup, a fixed order)
__global__ void __launch_bounds__(kBlock)
    k_sum_parts(int n, const double* __restrict__ part,
                DevStats* __restrict__ st) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += kBlock) v += part[i];
  __shared__ double ws[kBlock / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) s += ws[w];
    st->depth_sum = s;
  }
}

// FP32-bulk depth arrays hold s = h - max(H, 0) (Store<float>); the depth
// they give back to the host is s + max(H, 0) in FP64
__global__ void k_depth_from_eta(int n, const float* __restrict__ s,
                                 const float* __restrict__ H,
                                 double* __restrict__ h) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double Hi = (double)H[i];
    h[i] = (double)s[i] + (Hi > 0.0 ? Hi : 0.0);
  }
}

// -------------------------------------------------------------------------
// ensemble control.  The members of an ensemble run their pressure solves in
// lockstep cycles; each member leaves the cycles at its own convergence check
// and its result then becomes its logical iterate 0.  These records are only
// written by k_ens_begin and k_ens_check (one workgroup each).
// -------------------------------------------------------------------------
struct EnsMember {
  int active;              // takes part in the running solve
  int rot;                 // logical iterate buffer i is buffer (i + rot) % 3
  int sweeps[2];           // sweeps of the last solve of each stage
  int noconv;              // solves stopped by the sweep cap or a NaN measure
  double tol;              // convergence tolerance of the member
  double measure;          // measure at the end of the last solve
  long long sweeps_total;  // since the state was set
  long long solves_total;
};

// every member takes part in the solve about to start; sync (or null): the
// grid-barrier arrivals (sync[0]) and the 8 item counters (sync[2..9]) of a
// one-launch ensemble solve start from 0
__global__ void k_ens_begin(EnsMember* __restrict__ mem, int n,
                            unsigned long long* sync) {
  for (int g = threadIdx.x; g < n; g += blockDim.x) mem[g].active = 1;
  if (sync && threadIdx.x < 10 && threadIdx.x != 1) sync[threadIdx.x] = 0ull;
}

// Convergence check of one active member by one workgroup: the max of its
// per-tile measures of the iterate p^kc; the member stops when it is below
// its tolerance, when kc reached the sweep cap or when it is not finite, and
// its saved iterate p^kc (logical buffer `save`) becomes logical buffer 0.
// COH: every access to the measures and to the member's record is at device
// scope (the one-launch ensemble solve, where other XCDs read them next).
template <bool COH>
__device__ __forceinline__ int ens_ld(int* p) {
  if constexpr (COH)
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    return *p;
}
template <bool COH>
__device__ __forceinline__ void ens_st(int* p, int v) {
  if constexpr (COH)
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    *p = v;
}
template <bool COH>
__device__ __forceinline__ long long ens_ld(long long* p) {
  if constexpr (COH)
    return (long long)ld_agent_u64(reinterpret_cast<unsigned long long*>(p));
  else
    return *p;
}
template <bool COH>
__device__ __forceinline__ void ens_st(long long* p, long long v) {
  if constexpr (COH)
    st_agent_u64(reinterpret_cast<unsigned long long*>(p),
                 (unsigned long long)v);
  else
    *p = v;
}
template <bool COH>
__device__ __forceinline__ double ens_ld(double* p) {
  if constexpr (COH)
    return ld_agent(p);
  else
    return *p;
}
template <bool COH>
__device__ __forceinline__ void ens_st(double* p, double v) {
  if constexpr (COH)
    st_agent(p, v);
  else
    *p = v;
}

template <typename T, bool COH>
__device__ __forceinline__ void ens_check_body(const SweepArgs<T>& a,
                                               EnsMember& m, int kc, int kmax,
                                               int save, int stage,
                                               double* E_host,
                                               int* active_host, int g) {
  const double* part = a.part;
  const int nt = a.ntiles;
  double v = 0.0;
  for (int i = threadIdx.x; i < nt; i += blockDim.x) {
    double x;
    if constexpr (COH)
      x = ld_agent(part + i);
    else
      x = part[i];
    v = (x > v || x != x) ? x : v;
  }
  __shared__ double wmax[1024 / 64];  // any workgroup size
  v = wave_max(v);
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    v = wmax[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
      v = (wmax[w] > v || wmax[w] != wmax[w]) ? wmax[w] : v;
    const bool ok = v < ens_ld<COH>(&m.tol);
    const bool stop = ok || kc >= kmax || !(v == v) || isinf(v);
    if (stop) {
      ens_st<COH>(&m.rot, (ens_ld<COH>(&m.rot) + save) % 3);
      ens_st<COH>(&m.sweeps[stage], kc);
      ens_st<COH>(&m.measure, v);
      ens_st<COH>(&m.sweeps_total, ens_ld<COH>(&m.sweeps_total) + kc);
      ens_st<COH>(&m.solves_total, ens_ld<COH>(&m.solves_total) + 1);
      if (!ok) ens_st<COH>(&m.noconv, ens_ld<COH>(&m.noconv) + 1);
      ens_st<COH>(&m.active, 0);
    }
    if (E_host) {
      E_host[g] = v;
      active_host[g] = stop ? 0 : 1;
    }
  }
  __syncthreads();  // wmax is written again by the next check
}

// The check of every active member, one workgroup per member.  The measure
// and the active flag go to mapped host memory.
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_ens_check(const SweepArgs<T>* __restrict__ as,
                EnsMember* __restrict__ mem, int kc, int kmax, int save,
                int stage, double* __restrict__ E_host,
                int* __restrict__ active_host) {
  const int g = blockIdx.x;
  if (!mem[g].active) return;  // uniform over the workgroup
  ens_check_body<T, false>(as[g], mem[g], kc, kmax, save, stage, E_host,
                           active_host, g);
}

// After k_ens_check: the number of members still active goes to mapped host
// memory, then the check's sequence number (release at system scope).
__global__ void __launch_bounds__(kBlock)
    k_ens_publish(const EnsMember* __restrict__ mem, int n,
                  int* __restrict__ nactive_host, long long* seq_slot,
                  long long seq) {
  int c = 0;
  for (int g = threadIdx.x; g < n; g += blockDim.x) c += mem[g].active;
  __shared__ int cnt[kBlock / 64];
  for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o, 64);
  if ((threadIdx.x & 63) == 0) cnt[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += cnt[w];
    *nactive_host = tot;
    __threadfence_system();
    __hip_atomic_store(seq_slot, seq, __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// After a check: the members still active, in order, and the exclusive
// prefix of their sweep workgroup counts nb[] (one thread; a few hundred
// members at most).  The host forms the same total from the active flags it
// reads in mapped memory.
__global__ void k_ens_compact(const EnsMember* __restrict__ mem,
                              const int* __restrict__ nb, int n,
                              int* __restrict__ ids, int* __restrict__ pre) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int m = 0, acc = 0;
  for (int g = 0; g < n; ++g) {
    if (!mem[g].active) continue;
    ids[m] = g;
    pre[m] = acc;
    acc += nb[g];
    ++m;
  }
  pre[m] = acc;
}

// -------------------------------------------------------------------------
// kernel entry points: one grid, or a batch of grids in one launch.  A batch
// maps its workgroups onto the grids through an exclusive prefix sum of the
// per-grid workgroup counts (prefix[g] <= block < prefix[g+1]); every grid is
// processed by exactly the arithmetic of its single-grid launch.
// -------------------------------------------------------------------------
__device__ __forceinline__ int batch_grid(const int* __restrict__ prefix,
                                          int ngrids, int block) {
  int lo = 0, hi = ngrids - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= block) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <typename T, bool ONE_D>
__global__ void __launch_bounds__(kBlock) k_fv(FvArgs<T> a) {
  fv_body<T, ONE_D>(a, xcd_bid());
}
template <typename T, bool ONE_D>
__global__ void __launch_bounds__(kBlock)
    k_fv_batch(const FvArgs<T>* __restrict__ as, const int* __restrict__ pre,
               int ngrids) {
  const int bb = xcd_bid();
  int g = batch_grid(pre, ngrids, bb);
  fv_body<T, ONE_D>(as[g], bb - pre[g]);
}

template <typename T, bool ONE_D>
__global__ void __launch_bounds__(kBlock) k_break_cells(BreakCellsArgs<T> a) {
  break_cells_body<T, ONE_D>(a, xcd_bid());
}
template <typename T, bool ONE_D>
__global__ void __launch_bounds__(kBlock)
    k_break_cells_batch(const BreakCellsArgs<T>* __restrict__ as,
                        const int* __restrict__ pre, int ngrids) {
  const int bb = xcd_bid();
  int g = batch_grid(pre, ngrids, bb);
  break_cells_body<T, ONE_D>(as[g], bb - pre[g]);
}

template <typename T, bool ONE_D>
__global__ void __launch_bounds__(kBlock)
    k_break_corners(BreakCornersArgs<T> a) {
  break_corners_body<T, ONE_D>(a, xcd_bid());
}
template <typename T, bool ONE_D>
__global__ void __launch_bounds__(kBlock)
    k_break_corners_batch(const BreakCornersArgs<T>* __restrict__ as,
                          const int* __restrict__ pre, int ngrids) {
  const int bb = xcd_bid();
  int g = batch_grid(pre, ngrids, bb);
  break_corners_body<T, ONE_D>(as[g], bb - pre[g]);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_assemble2d(AssembleArgs<T> a) {
  assemble2d_body<T>(a, xcd_bid());
}
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_assemble2d_batch(const AssembleArgs<T>* __restrict__ as,
                       const int* __restrict__ pre, int ngrids) {
  const int bb = xcd_bid();
  int g = batch_grid(pre, ngrids, bb);
  assemble2d_body<T>(as[g], bb - pre[g]);
}

template <typename T, int B, int S, int M>
__global__ void __launch_bounds__(B)
    k_sweep_tb(SweepArgs<T> a, SweepLaunch L) {
  extern __shared__ double lds[];
  if (L.reduce && (int)blockIdx.x == a.nblocks()) {
    __shared__ double wmax[B / 64];
    double v = 0.0;
    for (int i = threadIdx.x; i < a.ntiles; i += B) {
      double x = a.part[i];
      v = (x > v || x != x) ? x : v;
    }
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double m = wmax[0];
      for (int w = 1; w < B / 64; ++w)
        m = (wmax[w] > m || wmax[w] != wmax[w]) ? wmax[w] : m;
      *L.E_host = check_measure(a.rmax, m);
      __threadfence_system();
      __hip_atomic_store(L.seq_slot, L.seq, __ATOMIC_RELEASE,
                         __HIP_MEMORY_SCOPE_SYSTEM);
    }
    return;
  }
  sweep_body<T, B, S, M>(a, L, (int)blockIdx.x, lds);
}
// batch: the launch covers the members ids[0..ngrids) (the members still
// active in the running solve, compacted after each check), members found
// inactive are skipped; the launch's buffer indices are logical and map to
// (index + rot) % 3 of each member.  Every member's workgroup count is a
// multiple of 8, so the local workgroup index keeps the XCD of the global one.
template <typename T, int B, int S, int M>
__global__ void __launch_bounds__(B)
    k_sweep_tb_batch(const SweepArgs<T>* __restrict__ as,
                     const int* __restrict__ ids, const int* __restrict__ pre,
                     int ngrids, const EnsMember* __restrict__ mem,
                     SweepLaunch L) {
  extern __shared__ double lds[];
  const int pos = batch_grid(pre, ngrids, (int)blockIdx.x);
  const int g = ids[pos];
  if (!mem[g].active) return;
  const int r = mem[g].rot;
  SweepLaunch Lg = L;
  Lg.iin = (L.iin + r) % 3;
  Lg.iout = (L.iout + r) % 3;
  Lg.isave = (L.isave + r) % 3;
  sweep_body<T, B, S, M>(as[g], Lg, (int)blockIdx.x - pre[pos], lds);
}

// -------------------------------------------------------------------------
// The lockstep solve of an ensemble in one cooperative launch: the launches
// of 8 sweeps over every member's tiles and the convergence checks between
// them become phases of one kernel, separated by grid barriers, so that the
// host takes no decision during a solve and a whole step is a fixed sequence
// of launches.  Every phase does the work of the launch it replaces, in the
// same order of blocks and checks, so that the members' iterates, sweep
// counts and measures are the same to the bit:
//   - a sweep phase: the workgroups take the (member, tile) items of the
//     members still active, from a table of those members that every
//     workgroup forms after each check.  Items are handed out as they are
//     asked for (an atomic counter per XCD class: workgroup w takes items
//     i = w mod 8 (mod 8), so that a tile keeps the XCD it has in the sweep
//     launches), which keeps the workgroups busy to the end of the phase
//     however the items' costs differ;
//   - a check phase: one workgroup per member still active.
// The iterate, the saved iterate, the per-tile measures and the member
// records are read and written at device scope: a phase reads what other
// XCDs wrote in the one before, once every workgroup has passed the barrier
// between them.  A barrier counts arrivals in one 64-bit word (zeroed before
// the launch); every wait is bounded and gives up through the flags word.
// -------------------------------------------------------------------------
struct EnsPersist {
  int kmax, ce, stage;        // sweep cap, sweeps per check, stage
  unsigned long long* bar;    // barrier arrivals (0 at the launch)
  unsigned long long* items;  // 8 item counters (0 at the launch)
  int* flags;                 // kFlagWaitBound when a wait gave up
  long long bound;            // polls before a wait gives up
};
constexpr int kEnsPersistMax = 1024;  // members of a one-launch solve

// two 1024-thread workgroups per CU, as the sweep launches have (64
// registers per thread)
template <typename T, int B, int S, int M>
__global__ void __launch_bounds__(B) __attribute__((amdgpu_waves_per_eu(8, 8)))
    k_ens_solve(const SweepArgs<T>* __restrict__ as,
                const int* __restrict__ pre, int L,
                EnsMember* __restrict__ mem, EnsPersist P) {
  extern __shared__ double lds[];
  // the members still active in order, the prefix of their items, and
  // every member's buffer rotation (the table of a compacted launch)
  __shared__ int s_ids[kEnsPersistMax], s_pre[kEnsPersistMax + 1];
  __shared__ int s_rot[kEnsPersistMax];
  __shared__ int s_give_up, s_nact, s_next;
  const int G = (int)gridDim.x, tid = (int)threadIdx.x;
  // this workgroup's XCD class and its item counter; every workgroup of a
  // class makes exactly one grab past the end of each phase, so the class's
  // counter advances by its items plus G / 8 per phase
  const int xc = (int)blockIdx.x & 7;
  unsigned long long* const ctr = P.items + xc;
  unsigned long long cbase = 0;
  auto grab = [&]() {
    return __hip_atomic_fetch_add(ctr, 1ull, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
  };
  if (tid == 0) s_give_up = 0;
  unsigned long long nbar = 0;
  // every workgroup's device-scope writes of the phase have completed
  // before any workgroup reads them in the next one
  auto barrier = [&]() {
    wait_memory();
    __syncthreads();
    if (tid == 0) {
      __hip_atomic_fetch_add(P.bar, 1ull, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
      const unsigned long long want = (nbar + 1) * (unsigned long long)G;
      long long it = 0;
      // (a negative bound gives up at once: the host asks for that path)
      while (ld_agent_u64(P.bar) < want || P.bound < 0) {
        if (++it > P.bound || ((it & 63) == 0 && gave_up(P.flags))) {
          s_give_up = 1;
          atomicOr(P.flags, kFlagWaitBound);
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    __syncthreads();
    ++nbar;
    return s_give_up == 0;
  };
  // the table, from the member records (every workgroup forms the same)
  auto table = [&]() {
    for (int g = tid; g < L; g += B) {
      s_ids[g] = ens_ld<true>(&mem[g].active);
      s_rot[g] = ens_ld<true>(&mem[g].rot);
    }
    __syncthreads();
    if (tid == 0) {
      int m = 0, acc = 0;
      for (int g = 0; g < L; ++g) {
        if (!s_ids[g]) continue;
        s_ids[m] = g;  // m <= g: read before written
        s_pre[m] = acc;
        acc += pre[g + 1] - pre[g];
        ++m;
      }
      s_pre[m] = acc;
      s_nact = m;
    }
    __syncthreads();
  };
  // the items of the active members (the prefix holds multiples of 8: the
  // items of a class are it = 8 j + xc, j < total / 8)
  auto sweeps = [&](const SweepLaunch& Lc) {
    const int nact = s_nact, total = s_pre[nact], per = total / 8;
    if (tid == 0) s_next = (int)(grab() - cbase);
    __syncthreads();
    int j = s_next;
    __syncthreads();
    while (j < per) {
      // the next item is asked for while this one is swept
      unsigned long long nx = 0;
      if (tid == 0) nx = grab();
      const int it = 8 * j + xc;
      int lo = 0, hi = nact - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_pre[mid] <= it) lo = mid; else hi = mid - 1;
      }
      const int g = s_ids[lo], r = s_rot[g];
      SweepLaunch Lg = Lc;
      Lg.iin = (Lc.iin + r) % 3;
      Lg.iout = (Lc.iout + r) % 3;
      Lg.isave = (Lc.isave + r) % 3;
      sweep_body<T, B, S, M, true>(as[g], Lg, it - s_pre[lo], lds);
      if (tid == 0) s_next = (int)(nx - cbase);
      __syncthreads();  // the LDS planes are filled again by the next item
      j = s_next;
      __syncthreads();
    }
    cbase += (unsigned long long)(per + G / 8);
  };
  const int ce = P.ce, kmax = P.kmax, stage = P.stage;
  int k = 0, cur = 0;
  table();
  for (;;) {
    const int save = (cur + 2) % 3, out = (cur + 1) % 3;
    const int kc = k;
    const int nsw = k >= kmax ? 0 : min(min(S, ce), kmax - k);
    sweeps(SweepLaunch{cur, out, save, k, nsw, 1, 0, nullptr, nullptr, 0});
    if (!barrier()) return;
    for (int i = (int)blockIdx.x; i < s_nact; i += G) {
      const int g = s_ids[i];
      ens_check_body<T, true>(as[g], mem[g], kc, kmax, save, stage, nullptr,
                              nullptr, g);
    }
    if (!barrier()) return;
    if (nsw > 0) {
      cur = out;
      k += nsw;
    }
    table();
    if (s_nact == 0) return;  // every member has stopped
    int other = 3 - cur - save;
    while (k % ce != 0 && k < kmax) {
      const int n2 = min(min(S, ce - k % ce), kmax - k);
      sweeps(SweepLaunch{cur, other, other, k, n2, 0, 0, nullptr, nullptr, 0});
      if (!barrier()) return;
      const int t = cur;
      cur = other;
      other = t;
      k += n2;
    }
  }
}

// -------------------------------------------------------------------------
// A whole relaxation solve in one launch, for grids whose tiles all fit
// the co-resident workgroups (one tile per workgroup; launched with no more
// workgroups than the device holds at once, cooperatively on request).  The sweeps,
// the schedule and the checks are those of k_sweep_tb and of the host loop
// that drives it: the same update of every corner in the same order of
// operations, blocks of sweeps cut at every check and at the sweep cap, and
// at each check the measure of eq. (32) of the iterate, so that the result
// and its sweep count are the same.  What changes is where the solve lives
// between blocks: each workgroup keeps the rows and the iterate of its
// region (its own corners and those within S of them) in registers for the
// whole solve, a thread holding a column segment of M points (the north and
// south neighbours inside the segment come from its registers, the rest
// through LDS), and only the points that other tiles own are refreshed
// between blocks of at most S sweeps.
//
// Exchange: after block e a tile writes its corners into exchange buffer
// (e + 1) % 2, each value as two 64-bit words that carry its upper and lower
// half beside the block's tag; a tile starts block e + 1 by reading the
// points it does not own from that buffer until both tags of each are those
// of block e + 1.  The words are agent-scope atomics (coherent across the
// XCDs' L2s without cache write-backs or invalidations), so no flag and no
// fence is needed.  Two buffers suffice: tile A reads tile B exactly when B
// reads A (each reads the corners within S of its own), so B overwrites
// buffer e % 2 (after block e + 1, whose start read A's block e + 1 values)
// only once A has finished block e and with it its reads of that buffer.
// Tags grow over the solver's life (the base is the block count of all
// earlier solves, the same on every tile), so no solve takes another's
// values.  On a periodic line the last corner is the first one again: it
// belongs to the tile of the first corner and is written with it into the
// result.
//
// Checks: each tile writes the measure of its corners into its slot of one
// of two slot arrays (by the parity of the check), as two tagged words like
// the exchange, and goes on with its block; after the block it reads every
// tile's slot until all carry the check's tag, and every workgroup takes
// the same decision from the same values.  (Two arrays suffice: a tile
// writes the slots of check c + 2 only after every tile has written those of
// c + 1, after its own reads of check c.)  The input iterate of a check is
// written to the result buffer, so that a stop leaves the result there.
//
// Every wait is bounded: a wait that reaches its bound, or that sees the
// give-up bit of another workgroup, sets that bit and ends its workgroup,
// and the host reports the failed solve.
// -------------------------------------------------------------------------
// position of an unwrapped corner index on a periodic line of n corners
__device__ __forceinline__ int cyc(int u, int n) {
  const int r = u % n;
  return r < 0 ? r + n : r;
}
struct PersistSync {
  unsigned long long* xch0;  // exchange buffers, 2 words per corner
  unsigned long long* xch1;
  unsigned* blocks;  // [0] blocks, [1] checks of all earlier solves (tag
                     // bases)
  unsigned long long* slots;  // per-tile measures: 2 arrays x ntiles x 2
                              // words
  int* flags;        // solver flags (kFlagWaitBound)
  DevStats* st;      // solve statistics (written by workgroup 0)
  long long bound;   // polls before a wait gives up
};

struct PersistLaunch {
  int iin, iout;        // initial iterate, result (different buffers)
  int kmax, ce, stage;  // sweep cap, sweeps per check, stage of the step
  int timed;            // the host times this launch: count its sweeps
  double tol;
};

// a value and its tag as the two words of the exchange
__device__ __forceinline__ unsigned long long xword(unsigned tag,
                                                    unsigned half) {
  return ((unsigned long long)tag << 32) | half;
}

// LDS planes of the one-launch solve.  The RW threads of a thread row hold
// M region rows of RW places; consecutive thread rows are a pitch apart
// that is congruent to RW modulo 32 places (256 bytes, one pass of the LDS
// banks), so that the lanes of a wave that run from the end of one thread
// row into the next read consecutive banks as lanes within a row do.
__host__ __device__ constexpr int persist_pitch(int M, int RW) {
  return M * RW + (((RW - M * RW) % 32) + 32) % 32;
}
// places before a plane's first thread row: the point below it is read
__host__ __device__ constexpr int persist_front(int M, int RW) {
  return persist_pitch(M, RW) - (M - 1) * RW + 1;
}
// places of one plane: the thread rows of all B threads, the point above
// the last one and the padding before the first
__host__ __device__ constexpr int persist_plane(int B, int M, int RW) {
  return persist_front(M, RW) + (B / RW + 1) * persist_pitch(M, RW) + RW + 1;
}
// LDS bytes of the one-launch solve: two FP64 planes
__host__ __device__ constexpr long persist_lds_bytes(int B, int M, int RW) {
  return 2L * 8 * persist_plane(B, M, RW);
}

// The exchange buffers through a buffer resource: a corner's two words
// {upper half, tag, lower half, tag} move as one 16-byte access at device
// scope (coherent across the XCDs' L2s); a torn access shows as differing
// tags and is read again.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kCoherent = 16;  // cache policy bits: device scope (sc1)
__device__ __forceinline__ __amdgpu_buffer_rsrc_t xrsrc(
    unsigned long long* p, long ncorn) {
  // raw (unformatted) buffer of 16 bytes per corner
  return __builtin_amdgcn_make_buffer_rsrc(p, 0, (int)(16 * ncorn),
                                           0x00020000);
}
__device__ __forceinline__ u32x4 xload(__amdgpu_buffer_rsrc_t r, int g) {
  return __builtin_amdgcn_raw_buffer_load_b128(r, g * 16, 0, kCoherent);
}
__device__ __forceinline__ void xstore(__amdgpu_buffer_rsrc_t r, int g,
                                       unsigned tag, double v) {
  const u32x4 w = {(unsigned)__double2hiint(v), tag,
                   (unsigned)__double2loint(v), tag};
  __builtin_amdgcn_raw_buffer_store_b128(w, r, g * 16, 0, kCoherent);
}

// kinds of a region point (pk: corner index << 5 | these bits; -1: none);
// kPkPub: an own corner that other tiles read (within S of the tile's edge)
constexpr int kPkOwn = 1, kPkRing = 2, kPkDupX = 4, kPkDupY = 8,
              kPkPub = 16, kPkShift = 5;

template <typename T, int B, int S, int M>
__global__ void __launch_bounds__(B)
    k_solve_persist(SweepArgs<T> a, PersistLaunch L, PersistSync Y) {
  extern __shared__ double lds[];
  __shared__ int give_up;
  __shared__ double wred[B / 64];
  __shared__ double om_s[kPersistOmega];
  const int ncx = a.ncx, ncy = a.ncy, BX = a.BX, BY = a.BY, ntx = a.ntx;
  const int ntiles = a.ntiles;
  const int tile = (int)blockIdx.x;  // the grid has exactly ntiles groups
  const int tid = (int)threadIdx.x;
  const int tx = tile % ntx, ty = tile / ntx;
  const int RW = BX + 2 * S, RH = BY + 2 * S;
  // the relaxation schedule in LDS (the host keeps nom <= kPersistOmega)
  for (int i = tid; i < a.nom; i += B) om_s[i] = a.omega[i];
  const int x0 = tx * BX - S, y0 = ty * BY - S;
  const bool px = (a.bc & kPerX) != 0, py = (a.bc & kPerY) != 0;
  // distinct corners of a line (on a periodic line the last one is the
  // first one again) and the corners this tile owns
  const int nlx = px ? ncx - 1 : ncx, nly = py ? ncy - 1 : ncy;
  const int ox0 = tx * BX, ox1 = min(ox0 + BX, nlx);
  const int oy0 = ty * BY, oy1 = min(oy0 + BY, nly);
  const int nseg = (RH + M - 1) / M;
  const int cx = tid % RW, ys = (tid / RW) * M;
  const bool active = tid < RW * nseg;
  // two LDS planes: the thread rows' M region rows of RW places each, a
  // bank-aligned pitch apart (rows past the region included), padded so
  // that the neighbours of any point are inside
  const int PT = persist_pitch(M, RW), PL = persist_plane(B, M, RW);
  double* L0 = lds + persist_front(M, RW);
  double* L1 = L0 + PL;
  const int lbase = (tid / RW) * PT + cx;
  if (tid == 0) give_up = 0;
  const unsigned base = ld_agent_u32(Y.blocks);
  const unsigned cbase = ld_agent_u32(Y.blocks + 1);
  const T* __restrict__ dgl = a.diag;
  const T* __restrict__ cE = a.cE;
  const T* __restrict__ cW = a.cW;
  const T* __restrict__ cN = a.cN;
  const T* __restrict__ cS = a.cS;
  const T* __restrict__ rhs = a.rhs;
  const double* __restrict__ p0 = a.p[L.iin];
  // rows and iterate of the thread's points (outside the domain, and
  // farther than S from the tile's corners: diag 1, the rest 0, and the
  // iterate stays 0); the rows widened to FP64 once (exact for FP32 rows)
  double dg[M], ce[M], cw[M], cn[M], cs[M], cr[M];
  double rdg[M], v[M];
  int pk[M];
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int y = ys + m;
    ce[m] = cw[m] = cn[m] = cs[m] = cr[m] = 0.0;
    dg[m] = 1.0;
    v[m] = 0.0;
    pk[m] = -1;
    if (active && y < RH) {
      const int ux = x0 + cx, uy = y0 + y;
      const int gx = px ? cyc(ux, nlx) : ux;
      const int gy = py ? cyc(uy, nly) : uy;
      if (ux >= ox0 - S && ux < ox1 + S && uy >= oy0 - S && uy < oy1 + S &&
          gx >= 0 && gx < ncx && gy >= 0 && gy < ncy) {
        const int g = gy * ncx + gx;
        v[m] = p0[g];
        dg[m] = (double)dgl[g];
        ce[m] = (double)cE[g];
        cw[m] = (double)cW[g];
        cn[m] = (double)cN[g];
        cs[m] = (double)cS[g];
        cr[m] = (double)rhs[g];
        if (ux >= ox0 && ux < ox1 && uy >= oy0 && uy < oy1) {
          const bool pub = ux - ox0 < S || ox1 - 1 - ux < S ||
                           uy - oy0 < S || oy1 - 1 - uy < S;
          pk[m] = (g << kPkShift) | kPkOwn | (pub ? kPkPub : 0) |
                  (px && gx == 0 ? kPkDupX : 0) |
                  (py && gy == 0 ? kPkDupY : 0);
        } else {
          pk[m] = (g << kPkShift) | kPkRing;
        }
      }
    }
  }
#pragma unroll
  for (int m = 0; m < M; ++m) rdg[m] = 1.0 / dg[m];
  // a point's distance to the region's border (sweep t updates the points
  // farther than t from it; -1: no point), from its column's and its row's
  const int distx = active ? min(cx, RW - 1 - cx) : -1;
  auto dist = [&](int m) {
    const int y = ys + m;
    return y < RH ? min(distx, min(y, RH - 1 - y)) : -1;
  };
  double* const res = a.p[L.iout];
  const int nom = a.nom, cev = L.ce, kmax = L.kmax;
  const bool resid = a.rmax != nullptr;
  int k = 0, nchk = 0, e = 0;
  for (;;) {
    const bool check = (k % cev) == 0 || k >= kmax;
    const int nsw = k >= kmax ? 0 : min(min(S, cev - k % cev), kmax - k);
    if (e > 0) {
      // the points other tiles own, as those tiles left them after block e
      const unsigned want = base + (unsigned)e;
      const __amdgpu_buffer_rsrc_t X =
          xrsrc((e & 1) ? Y.xch1 : Y.xch0, (long)ncx * ncy);
      u32x4 w[M];
#pragma unroll
      for (int m = 0; m < M; ++m) {  // all loads in flight at once
        w[m] = u32x4{0u, want, 0u, want};
        if (pk[m] >= 0 && (pk[m] & kPkRing))
          w[m] = xload(X, pk[m] >> kPkShift);
      }
#pragma unroll
      for (int m = 0; m < M; ++m) {
        if (pk[m] >= 0 && (pk[m] & kPkRing)) {
          long long it = 0;
          while (w[m].y != want || w[m].w != want || Y.bound < 0) {
            if (++it > Y.bound || ((it & 63) == 0 && gave_up(Y.flags))) {
              give_up = 1;
              break;
            }
            __builtin_amdgcn_s_sleep(2);
            asm volatile("" ::: "memory");  // a new load every poll
            w[m] = xload(X, pk[m] >> kPkShift);
          }
          v[m] = __hiloint2double((int)w[m].x, (int)w[m].z);
        }
      }
      __syncthreads();
      if (give_up) {
        if (tid == 0) atomicOr(Y.flags, kFlagWaitBound);
        return;
      }
    }
    double emax = 0.0;
    const int iters = nsw > 0 ? nsw : 1;
    // one sweep over the thread's points from LDS plane Lb; CHK: the first
    // sweep of a check, which also takes the measure of the own points and
    // writes their input iterate to the result buffer; UPD: update
    auto relax = [&](auto chk, double* Lb, double om, int t, bool upd) {
      constexpr bool CHK = decltype(chk)::value;
      double pE[M], pW[M];
#pragma unroll
      for (int m = 0; m < M; ++m) {
        pE[m] = Lb[lbase + m * RW + 1];
        pW[m] = Lb[lbase + m * RW - 1];
      }
      const double pTop = Lb[lbase + PT];  // the next thread row's first
      // the input value of the point below: the previous thread row's last
      double below = Lb[lbase - PT + (M - 1) * RW];
#pragma unroll
      for (int m = 0; m < M; ++m) {
        const double pc = v[m];
        const double pN = (m + 1 < M) ? v[m + 1] : pTop;
        const double pS = below;
        below = pc;
        // a wave none of whose lanes updates (or, at a check, measures)
        // this point skips it
        const bool live = dist(m) > t;
        if (!__any((CHK || upd) && live)) continue;
        double Ap = dg[m] * pc;
        Ap = fma(ce[m], pE[m], Ap);
        Ap = fma(cw[m], pW[m], Ap);
        Ap = fma(cn[m], pN, Ap);
        Ap = fma(cs[m], pS, Ap);
        const double rr = cr[m] - Ap;
        const double rd = rr * rdg[m];
        const double pn = fma(om, rd, pc);
        if constexpr (CHK) {
          if (pk[m] >= 0 && (pk[m] & kPkOwn)) {
            const double ar = check_term(resid, rr, rdg[m]);
            emax = (ar > emax || ar != ar) ? ar : emax;
            // the result buffer is read after the launch only
            const int g = pk[m] >> kPkShift;
            res[g] = pc;
            if (pk[m] & kPkDupX) res[g + ncx - 1] = pc;
            if (pk[m] & kPkDupY) res[g + (ncy - 1) * ncx] = pc;
            if ((pk[m] & (kPkDupX | kPkDupY)) == (kPkDupX | kPkDupY))
              res[g + (ncy - 1) * ncx + ncx - 1] = pc;
          }
        }
        v[m] = (upd && live) ? pn : pc;
      }
    };
#pragma unroll
    for (int t = 0; t < S; ++t) {
      if (t >= iters) break;
      double* Lb = (t & 1) ? L1 : L0;
#pragma unroll
      for (int m = 0; m < M; ++m) Lb[lbase + m * RW] = v[m];
      __syncthreads();
      const double om = om_s[(k + t) % nom];
      if (t == 0 && check)
        relax(std::true_type{}, Lb, om, t, nsw > 0);
      else
        relax(std::false_type{}, Lb, om, t, true);
      if (t == 0 && check) {
        const double w = wave_max(emax);
        if ((tid & 63) == 0) wred[tid >> 6] = w;
        __syncthreads();
        if (tid == 0) {
          double mx = wred[0];
          for (int i = 1; i < B / 64; ++i)
            mx = (wred[i] > mx || wred[i] != wred[i]) ? wred[i] : mx;
          const unsigned tag = cbase + (unsigned)nchk + 1u;
          unsigned long long* sl =
              Y.slots + 2 * ((size_t)(nchk & 1) * ntiles + tile);
          st_agent_u64(sl, xword(tag, (unsigned)__double2hiint(mx)));
          st_agent_u64(sl + 1, xword(tag, (unsigned)__double2loint(mx)));
        }
      }
    }
    if (nsw > 0) {
      // publish the tile's corners that others read, after block e
      const unsigned tag = base + (unsigned)e + 1u;
      const __amdgpu_buffer_rsrc_t X =
          xrsrc(((e + 1) & 1) ? Y.xch1 : Y.xch0, (long)ncx * ncy);
#pragma unroll
      for (int m = 0; m < M; ++m)
        if (pk[m] >= 0 && (pk[m] & kPkPub))
          xstore(X, pk[m] >> kPkShift, tag, v[m]);
    }
    if (check) {
      // every tile's measure of this check
      const unsigned want = cbase + (unsigned)nchk + 1u;
      unsigned long long* sl = Y.slots + 2 * (size_t)(nchk & 1) * ntiles;
      double w = 0.0;
      for (int i = tid; i < ntiles; i += B) {
        unsigned long long w0 = ld_agent_u64(sl + 2 * i);
        unsigned long long w1 = ld_agent_u64(sl + 2 * i + 1);
        long long it = 0;
        while ((unsigned)(w0 >> 32) != want || (unsigned)(w1 >> 32) != want ||
               Y.bound < 0) {
          if (++it > Y.bound || ((it & 63) == 0 && gave_up(Y.flags))) {
            give_up = 1;
            break;
          }
          __builtin_amdgcn_s_sleep(2);
          w0 = ld_agent_u64(sl + 2 * i);
          w1 = ld_agent_u64(sl + 2 * i + 1);
        }
        const double x = __hiloint2double((int)(unsigned)w0, (int)(unsigned)w1);
        w = (x > w || x != x) ? x : w;
      }
      __syncthreads();
      if (give_up) {
        if (tid == 0) atomicOr(Y.flags, kFlagWaitBound);
        return;
      }
      w = wave_max(w);
      if ((tid & 63) == 0) wred[tid >> 6] = w;
      __syncthreads();
      double E = wred[0];
      for (int i = 1; i < B / 64; ++i)
        E = (wred[i] > E || wred[i] != wred[i]) ? wred[i] : E;
      E = check_measure(a.rmax, E);
      ++nchk;
      if (E < L.tol || k >= kmax) {
        if (tile == 0 && tid == 0) {
          DevStats* d = Y.st;
          d->sweeps[L.stage] = k;
          d->measure = E;
          d->sweeps_total += k;
          d->solves_total += 1;
          if (!(E < L.tol)) d->noconv += 1;
          if (L.timed) d->prof_sweeps += k;
          // blocks published and checks made by every tile: the next
          // solve's tag bases
          Y.blocks[0] = base + (unsigned)(e + (nsw > 0 ? 1 : 0));
          Y.blocks[1] = cbase + (unsigned)nchk;
        }
        return;
      }
      __syncthreads();  // wred is written again at the next check
    }
    k += nsw;
    e += 1;
  }
}

template <typename T, bool ONE_D, bool COMBINE>
__global__ void __launch_bounds__(kBlock) k_correct(CorrectArgs<T> a) {
  correct_body<T, ONE_D, COMBINE>(a, xcd_bid());
}
// batch: the pressure of member g is its logical iterate 0, buffer rot[g]
template <typename T, bool ONE_D, bool COMBINE>
__global__ void __launch_bounds__(kBlock)
    k_correct_batch(const CorrectArgs<T>* __restrict__ as,
                    const int* __restrict__ pre, int ngrids,
                    const SweepArgs<T>* __restrict__ sw,
                    const EnsMember* __restrict__ mem) {
  const int bb = xcd_bid();
  int g = batch_grid(pre, ngrids, bb);
  CorrectArgs<T> a = as[g];
  if (a.have_p) a.p = sw[g].p[mem[g].rot];
  correct_body<T, ONE_D, COMBINE>(a, bb - pre[g]);
}

template <typename T, bool ONE_D>
__global__ void __launch_bounds__(kBlock) k_lambda(LambdaArgs<T> a) {
  lambda_body<T, ONE_D>(a, xcd_bid());
}
template <typename T, bool ONE_D>
__global__ void __launch_bounds__(kBlock)
    k_lambda_batch(const LambdaArgs<T>* __restrict__ as,
                   const int* __restrict__ pre, int ngrids) {
  const int bb = xcd_bid();
  int g = batch_grid(pre, ngrids, bb);
  lambda_body<T, ONE_D>(as[g], bb - pre[g]);
}

__global__ void __launch_bounds__(kBlock) k_finalize_dt(FinalizeArgs a) {
  finalize_body(a);
}
// batch: one workgroup per grid
__global__ void __launch_bounds__(kBlock)
    k_finalize_dt_batch(const FinalizeArgs* __restrict__ as) {
  finalize_body(as[blockIdx.x]);
}

}  // namespace nh
