// nhswe.hip -- host orchestration and C ABI of the non-hydrostatic
// shallow-water time stepper for gfx950 (see include/nhswe.h).
//
// One step = two projection-correction stages (TVD-RK2, Section 6) and the
// device-side CFL reduction.  Each stage launches, on the solver's stream:
//   k_fv                                  finite-volume update (eq. 20, 30)
//   k_break_cells, k_break_corners        breaking terms (Section 3), if on
//   k_assemble2d | k_assemble1d           pressure system (eq. 37-41, 43)
//   k_sweep x K | k_thomas                solve (eq. 32) / Thomas (1D)
//   k_correct_cells, k_correct_corners    correction (eq. 36, 28, 41)
// The second stage's correction also forms the Runge-Kutta average and the
// CFL measure of the new state; k_finalize_dt turns it into the next dt.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "../../include/nhswe.h"
#include "kernels.hpp"
#include "adjoint.hpp"

namespace {

thread_local std::string g_err;

// Every failing call ends here.  A failed HIP call also stays the thread's
// "last error" in the runtime until someone reads it; it is read here, so
// that the caller's next check (torch's, after its next launch) does not
// report the library's failure as its own.
nh_status fail(nh_status st, const std::string& msg) {
  g_err = msg;
  (void)hipGetLastError();
  return st;
}

#define HIP_TRY(expr)                                                        \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess)                                                    \
      return fail(NH_EDEVICE, std::string(#expr) + ": " +                    \
                                  hipGetErrorString(e_));                    \
  } while (0)

inline unsigned nblocks(long n) {
  return (unsigned)((n + nh::kBlock - 1) / nh::kBlock);
}

// convergence measures published by the device to mapped host memory
struct HostSlot {
  long long seq;
  double E[1];
};

// Per-phase device timing: event pairs recorded on the stream and read
// lazily at the next synchronisation, so that timing never stalls the device.
struct ProfPool {
  bool on = false;
  // 1: every phase and every back-to-back sweep batch; n >= 2: only the
  // sweep batch of one cycle in n (each event pair stalls the queue for a
  // few microseconds, ~13 % of a step when every phase is timed)
  int sample = 1;
  long long nbatch = 0;
  long long nsolve = 0;  // one-launch solves seen (kind 5 samples by step)
  struct Mark {
    hipEvent_t a = nullptr, b = nullptr;
    int kind = 0;         // 0 fv, 1 assembly, 2 solve, 3 correction,
                          // 4 sweep launches, 5 one-launch solves
    long long count = 0;  // launches
    double work = 0.0;    // sweeps: corner-sweeps done by those launches
  };
  std::vector<Mark> marks;
  size_t used = 0;
  nh_profile_t pr{};

  // open an interval of the given kind on the stream (or -1)
  long open(hipStream_t st, int kind) {
    if (!on) return -1;
    if (sample > 1 && kind == 5) {
      if ((nsolve++ / 2) % sample != 0) return -1;
    } else if (sample > 1 && (kind != 4 || (nbatch++ % sample) != 0)) {
      return -1;
    }
    if (used == marks.size()) {
      Mark m;
      if (hipEventCreate(&m.a) != hipSuccess) return -1;
      if (hipEventCreate(&m.b) != hipSuccess) {
        hipEventDestroy(m.a);
        return -1;
      }
      marks.push_back(m);
    }
    Mark& m = marks[used];
    m.kind = kind;
    m.count = 0;
    m.work = 0.0;
    if (hipEventRecord(m.a, st) != hipSuccess) return -1;
    return (long)used++;
  }
  void close(hipStream_t st, long id, long long count, double work = 0.0) {
    if (id < 0) return;
    marks[id].count = count;
    marks[id].work = work;
    (void)hipEventRecord(marks[id].b, st);
  }
  // accumulate every closed interval (the stream has been synchronised)
  void flush() {
    for (size_t i = 0; i < used; ++i) {
      Mark& m = marks[i];
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, m.a, m.b) != hipSuccess) continue;
      switch (m.kind) {
        case 0: pr.fv_ms += ms; pr.fv_launches += m.count; break;
        case 1: pr.assemble_ms += ms; pr.assemble_launches += m.count; break;
        case 2: pr.solve_ms += ms; pr.solve_launches += m.count; break;
        case 3: pr.correct_ms += ms; pr.correct_launches += m.count; break;
        case 4:
          pr.sweep_kernel_ms += ms;
          pr.sweep_kernel_launches += m.count;
          pr.sweep_kernel_sweeps += m.count * nh::kSweepS;
          pr.sweep_kernel_corner_sweeps += m.work;
          break;
        case 5:
          pr.solve_kernel_ms += ms;
          pr.solve_kernel_launches += m.count;
          break;
      }
    }
    used = 0;
  }
  void release() {
    for (auto& m : marks) {
      if (m.a) hipEventDestroy(m.a);
      if (m.b) hipEventDestroy(m.b);
    }
    marks.clear();
    used = 0;
  }
};

}  // namespace

struct AdjWork;
void adj_release(AdjWork* w);  // adjoint work space (adjoint_impl.hpp)

struct nh_solver {
  nh_grid grid{};
  nh_params par{};
  std::vector<double> omega;
  int nom = 1;             // relaxation factors in the schedule
  bool one_d = false;
  bool fp32 = false;
  size_t esize = 8;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;          // HIP device current at nh_create
  long ncell = 0, ncorn = 0;

  // device buffers (element type double or float, see esize)
  void *H = nullptr, *h = nullptr, *q1 = nullptr, *q2 = nullptr;   // U^n
  void *hs = nullptr, *q1s = nullptr, *q2s = nullptr;              // U*
  void* hs_cur = nullptr;  // h* of the running stage (hs or h1)
  void *q1b = nullptr, *q2b = nullptr, *rw = nullptr;              // breaking
  void *h1 = nullptr, *q11 = nullptr, *q21 = nullptr;              // U^(1)
  void *w = nullptr, *ws = nullptr, *w1 = nullptr;                 // corners
  void* wadv = nullptr;  // w carried by the flow (w_advection)
  // FP32 bulk: the bathymetry as the caller gave it (FP64), against which a
  // host depth becomes the stored s = h - max(H, 0) (a lake at rest gets
  // eta = 0 exactly; against the FP32 bathymetry it would get the rounding
  // of H)
  std::vector<double> H_host;
  void *pa = nullptr, *pb = nullptr, *pc = nullptr;  // p (FP64, both modes)
  int pcur = 0;                            // index of the current iterate
  void *cdiag = nullptr, *cE = nullptr, *cW = nullptr, *cN = nullptr,
       *cS = nullptr, *crhs = nullptr;
  double *thomas_cp = nullptr, *thomas_dp = nullptr;
  double *thomas_bb = nullptr, *thomas_z = nullptr;  // cyclic (periodic 1D)
  void *stage_buf = nullptr;   // FP64 staging for host copies
  // generation/absorption zones: weights and targets (bulk type; p* FP64)
  bool relax_on = false;
  void *rm_c = nullptr, *rt_h = nullptr, *rt_q1 = nullptr, *rt_q2 = nullptr,
       *rm_k = nullptr, *rt_w = nullptr;
  double* rt_p = nullptr;
  // device scalars
  double* dt = nullptr;
  double* lampart = nullptr;             // per-block CFL measures
  double* part = nullptr;                // per-tile convergence measures
  nh::DevStats* dstats = nullptr;        // t, dt of the last step, steps
  HostSlot* slot = nullptr;              // mapped host memory (measure)
  HostSlot* slot_dev = nullptr;          // its device address
  double* E_dev = nullptr;               // = &slot_dev->E[0]
  double** part_list = nullptr;          // device: {part}
  int* ntiles_list = nullptr;            // device: {ntiles}
  long long seq = 0;
  int solve_launches_last = 0;
  double* omega_dev = nullptr;
  int tbx = 32, tby = 32, ntx = 1, nty = 1;  // sweep tiles
  int sweep_m = nh::kSweepM;  // region points per thread of the sweep
  // one cooperative launch per solve (k_solve_persist): its tiles and the
  // counters and slots its workgroups exchange through
  bool persist = false;
  int ptbx = 0, ptby = 0, pntx = 0, pnty = 0;
  size_t plds = 0;
  unsigned long long* p_xch = nullptr;  // 2 buffers x 2 words per corner
  unsigned* p_bar = nullptr;  // tag bases: [0] blocks, [1] checks
  unsigned long long* p_slots = nullptr;  // 2 x tiles x 2 words
  long long noconv_seen = 0;  // capped solves already reported
  double* rhs_max = nullptr;  // max |rhs| of the system (solve_norm 1)
  double* clamped = nullptr;
  int* flags = nullptr;
  // host mirrors
  void* pbuf(int i) { return i == 0 ? pa : (i == 1 ? pb : pc); }
  void* pcur_ptr() { return pbuf(pcur); }
  bool have_state = false, have_H = false;
  nh_stats st{};
  ProfPool prof;
  // recording of a forward run for the adjoint: the pressure of each stage
  // is copied here after its solve when set
  double* tape_p[2] = {nullptr, nullptr};
  struct AdjWork* adj = nullptr;
  int64_t adj_sweeps_last = 0;  // transposed-solve sweeps of the last run

  std::vector<void*> allocs;
};

namespace {

nh_status dalloc(nh_solver* s, void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();  // not left for the caller's next check
    *p = nullptr;
    return fail(NH_ENOMEM, "hipMalloc failed");
  }
  s->allocs.push_back(*p);
  hipMemsetAsync(*p, 0, bytes, s->stream);
  return NH_OK;
}

// copy a host FP64 array into a device array of the solver's type
nh_status upload(nh_solver* s, void* dst, const double* src, long n) {
  if (!s->fp32) {
    HIP_TRY(hipMemcpyAsync(dst, src, n * sizeof(double),
                           hipMemcpyHostToDevice, s->stream));
  } else {
    HIP_TRY(hipMemcpyAsync(s->stage_buf, src, n * sizeof(double),
                           hipMemcpyHostToDevice, s->stream));
    hipLaunchKernelGGL((nh::k_convert<float, double>), dim3(nblocks(n)),
                       dim3(nh::kBlock), 0, s->stream, (int)n,
                       (const double*)s->stage_buf, (float*)dst);
  }
  HIP_TRY(hipStreamSynchronize(s->stream));
  return NH_OK;
}

nh_status download(nh_solver* s, double* dst, const void* src, long n) {
  if (!s->fp32) {
    HIP_TRY(hipMemcpyAsync(dst, src, n * sizeof(double),
                           hipMemcpyDeviceToHost, s->stream));
  } else {
    hipLaunchKernelGGL((nh::k_convert<double, float>), dim3(nblocks(n)),
                       dim3(nh::kBlock), 0, s->stream, (int)n,
                       (const float*)src, (double*)s->stage_buf);
    HIP_TRY(hipMemcpyAsync(dst, s->stage_buf, n * sizeof(double),
                           hipMemcpyDeviceToHost, s->stream));
  }
  HIP_TRY(hipStreamSynchronize(s->stream));
  return NH_OK;
}

// host FP64 depths into a depth array of the solver.  FP32 bulk stores
// s = h - max(H, 0), formed in FP64 against the bathymetry as the caller
// gave it (which must be set first) and rounded once: a lake at rest gets
// eta = 0 over water and stays at rest to the bit; a dry cell gets -max(H,0).
nh_status upload_depth(nh_solver* s, void* dst, const double* h, long n) {
  if (!s->fp32) return upload(s, dst, h, n);
  if ((long)s->H_host.size() != n)
    return fail(NH_ESTATE, "set the bathymetry first");
  std::vector<double> sv(n);
  for (long i = 0; i < n; ++i) {
    const double Hi = s->H_host[i];
    sv[i] = h[i] - (Hi > 0.0 ? Hi : 0.0);
  }
  return upload(s, dst, sv.data(), n);
}

// a depth array of the solver to host FP64 depths
nh_status download_depth(nh_solver* s, double* h, const void* src, long n) {
  if (!s->fp32) return download(s, h, src, n);
  hipLaunchKernelGGL(nh::k_depth_from_eta, dim3(nblocks(n)), dim3(nh::kBlock),
                     0, s->stream, (int)n, (const float*)src,
                     (const float*)s->H, (double*)s->stage_buf);
  HIP_TRY(hipMemcpyAsync(h, s->stage_buf, n * sizeof(double),
                         hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return NH_OK;
}

// ---------------------------------------------------------------------------
// typed launch helpers
// ---------------------------------------------------------------------------
// Pointers of one projection-correction stage: stage 0 maps U^n to U^(1)
// (its h* is U^(1)'s depth, kept in hs), stage 1 maps U^(1) to U^(2) and
// averages it with U^n in place.
struct StagePlan {
  void *Vh, *Vq1, *Vq2, *w_in;  // stage input
  void* hs_cur;                 // h* of the stage
  void *qa, *qb, *wst;          // discharges and w fed to the pressure system
  void *oq1, *oq2, *w_out;      // stage output (stage 1: U^n in place)
  bool combine;
};

StagePlan stage_plan(const nh_solver* s, int idx) {
  StagePlan P;
  if (idx == 0) {
    P.Vh = s->h; P.Vq1 = s->q1; P.Vq2 = s->q2; P.w_in = s->w;
    P.hs_cur = s->hs;
    P.oq1 = s->q11; P.oq2 = s->q21; P.w_out = s->w1;
  } else {
    P.Vh = s->hs; P.Vq1 = s->q11; P.Vq2 = s->q21; P.w_in = s->w1;
    P.hs_cur = s->h1;
    P.oq1 = nullptr; P.oq2 = nullptr; P.w_out = s->w;
  }
  if (s->par.breaking_on) {
    P.qa = s->q1b; P.qb = s->q2b; P.wst = s->ws;
  } else {
    P.qa = s->q1s; P.qb = s->q2s; P.wst = P.w_in;
  }
  P.combine = idx == 1;
  return P;
}

// A five-point system on the corners of the grid and the three buffers of
// its relaxation iterate: the solver's own pressure system, or the transposed
// system of the adjoint.
struct SysView {
  void *diag, *cE, *cW, *cN, *cS, *rhs;
  double* p[3];
};

inline SysView forward_system(const nh_solver* s) {
  return SysView{s->cdiag, s->cE, s->cW, s->cN, s->cS, s->crhs,
                 {(double*)s->pa, (double*)s->pb, (double*)s->pc}};
}

// boundary mask of the kernels: open sides and periodic directions
inline int bc_mask(const nh_solver* s) {
  const auto& pr = s->par;
  return pr.open_sides | ((pr.periodic & 1) ? nh::kPerX : 0) |
         ((!s->one_d && (pr.periodic & 2)) ? nh::kPerY : 0);
}

// kernel arguments of one grid, shared by the single-grid launches and the
// ensemble's batched launches
template <typename T>
struct Args {
  static T* P(void* p) { return static_cast<T*>(p); }

  static nh::FvArgs<T> fv(const nh_solver* s, const StagePlan& S) {
    const auto& g = s->grid;
    const auto& pr = s->par;
    return nh::FvArgs<T>{g.nx, g.ny, (T)g.dx, (T)g.dy, (T)pr.g,
                         (T)pr.delta, (T)pr.dry_eps, P(S.Vh), P(S.Vq1),
                         P(S.Vq2), P(s->H), s->dt, P(S.hs_cur), P(s->q1s),
                         P(s->q2s), s->clamped,
                         (T)(pr.g * pr.manning * pr.manning), bc_mask(s)};
  }
  static nh::BreakCellsArgs<T> break_cells(const nh_solver* s,
                                           const StagePlan& S) {
    const auto& g = s->grid;
    const auto& pr = s->par;
    return nh::BreakCellsArgs<T>{g.nx, g.ny, (T)g.dx, (T)g.dy, (T)pr.g,
                                 (T)pr.delta, (T)pr.dry_eps, (T)pr.b1,
                                 P(S.hs_cur), P(s->q1s), P(s->q2s), P(s->H),
                                 s->dt, P(s->q1b), P(s->q2b), P(s->rw),
                                 bc_mask(s)};
  }
  static nh::BreakCornersArgs<T> break_corners(const nh_solver* s,
                                               const StagePlan& S) {
    return nh::BreakCornersArgs<T>{s->grid.nx, s->grid.ny, (T)s->par.delta,
                                   P(S.hs_cur), P(s->rw), P(s->H), s->dt,
                                   P(S.w_in), P(s->ws), bc_mask(s)};
  }
  static nh::AssembleArgs<T> assemble(const nh_solver* s, const StagePlan& S) {
    const auto& g = s->grid;
    return nh::AssembleArgs<T>{g.nx, g.ny, (T)g.dx, (T)g.dy, P(S.hs_cur),
                               P(S.qa), P(S.qb), P(s->H), P(S.wst), s->dt,
                               P(s->cdiag), P(s->cE), P(s->cW), P(s->cN),
                               P(s->cS), P(s->crhs), bc_mask(s),
                               s->dstats ? &s->dstats->nondom_run : nullptr};
  }
  static nh::SweepArgs<T> sweep(const nh_solver* s) {
    return sweep(s, forward_system(s));
  }
  static nh::SweepArgs<T> sweep(const nh_solver* s, const SysView& V) {
    nh::SweepArgs<T> a;
    a.ncx = s->grid.nx + 1;
    a.ncy = s->grid.ny + 1;
    a.BX = s->tbx;
    a.BY = s->tby;
    a.ntx = s->ntx;
    a.ntiles = s->ntx * s->nty;
    a.bc = bc_mask(s);
    a.diag = P(V.diag);
    a.cE = P(V.cE);
    a.cW = P(V.cW);
    a.cN = P(V.cN);
    a.cS = P(V.cS);
    a.rhs = P(V.rhs);
    a.p[0] = V.p[0];
    a.p[1] = V.p[1];
    a.p[2] = V.p[2];
    a.omega = s->omega_dev;
    a.nom = s->nom;
    a.part = s->part;
    a.rmax = s->par.solve_norm ? s->rhs_max : nullptr;
    return a;
  }
  // p: the solved pressure (ignored when the system is hydrostatic)
  static nh::CorrectArgs<T> correct(const nh_solver* s, const StagePlan& S,
                                    const void* p) {
    const auto& g = s->grid;
    const auto& pr = s->par;
    return nh::CorrectArgs<T>{g.nx, g.ny, (T)g.dx, (T)g.dy, (T)pr.g,
                              (T)pr.delta, (T)pr.dry_eps,
                              s->par.nh_on ? 1 : 0, P(S.hs_cur), P(S.qa),
                              P(S.qb), P(s->H), P(S.wst),
                              (const double*)(p ? p : s->pa), s->dt,
                              P(S.oq1), P(S.oq2), P(S.w_out), P(s->h),
                              P(s->q1), P(s->q2), s->lampart, s->flags,
                              s->relax_on ? P(s->rm_c) : nullptr, P(s->rt_h),
                              P(s->rt_q1), P(s->rt_q2),
                              s->relax_on ? P(s->rm_k) : nullptr,
                              P(s->rt_w), bc_mask(s)};
  }
  static nh::LambdaArgs<T> lambda(const nh_solver* s) {
    const auto& g = s->grid;
    const auto& pr = s->par;
    return nh::LambdaArgs<T>{g.nx, g.ny, (T)g.dx, (T)g.dy, (T)pr.g,
                             (T)pr.delta, (T)pr.dry_eps, P(s->h), P(s->q1),
                             P(s->q2), P(s->H), s->lampart};
  }
};

// end of a step (with_stats) or of set_state: dt from the CFL measures
inline nh::FinalizeArgs finalize_args(const nh_solver* s, bool with_stats) {
  if (with_stats)
    return nh::FinalizeArgs{s->par.cfl, s->par.fixed_dt, s->lampart,
                            (int)nblocks(std::max(s->ncell, s->ncorn)), s->dt,
                            s->flags, s->dstats};
  return nh::FinalizeArgs{s->par.cfl, 0, s->lampart, (int)nblocks(s->ncell),
                          s->dt, s->flags, nullptr};
}

inline size_t sweep_lds_bytes(int bx, int by) {
  return 2 * sizeof(double) * (bx + 2 * nh::kSweepS) * (by + 2 * nh::kSweepS);
}

template <typename T>
struct Launch {
  static T* P(void* p) { return static_cast<T*>(p); }

  static void fv(nh_solver* s, const StagePlan& S) {
    auto a = Args<T>::fv(s, S);
    if (s->one_d)
      hipLaunchKernelGGL((nh::k_fv<T, true>), dim3(a.nblocks()),
                         dim3(nh::kBlock), 0, s->stream, a);
    else
      hipLaunchKernelGGL((nh::k_fv<T, false>), dim3(a.nblocks()),
                         dim3(nh::kBlock), 0, s->stream, a);
  }

  static void advect_w(nh_solver* s, const StagePlan& S, void* w_out) {
    const auto& g = s->grid;
    const auto& pr = s->par;
    nh::AdvectWArgs<T> a{g.nx, g.ny, (T)g.dx, (T)g.dy, (T)pr.delta,
                         (T)pr.dry_eps, P(S.Vh), P(S.Vq1), P(S.Vq2), P(s->H),
                         P(S.w_in), s->dt, P(w_out), bc_mask(s)};
    if (s->one_d)
      hipLaunchKernelGGL((nh::k_advect_w<T, true>), dim3(a.nblocks(true)),
                         dim3(nh::kBlock), 0, s->stream, a);
    else
      hipLaunchKernelGGL((nh::k_advect_w<T, false>), dim3(a.nblocks(false)),
                         dim3(nh::kBlock), 0, s->stream, a);
  }

  static void breaking(nh_solver* s, const StagePlan& S) {
    auto c = Args<T>::break_cells(s, S);
    auto k = Args<T>::break_corners(s, S);
    if (s->one_d) {
      hipLaunchKernelGGL((nh::k_break_cells<T, true>), dim3(c.nblocks()),
                         dim3(nh::kBlock), 0, s->stream, c);
      hipLaunchKernelGGL((nh::k_break_corners<T, true>),
                         dim3(k.nblocks(true)), dim3(nh::kBlock), 0,
                         s->stream, k);
    } else {
      hipLaunchKernelGGL((nh::k_break_cells<T, false>), dim3(c.nblocks()),
                         dim3(nh::kBlock), 0, s->stream, c);
      hipLaunchKernelGGL((nh::k_break_corners<T, false>),
                         dim3(k.nblocks(false)), dim3(nh::kBlock), 0,
                         s->stream, k);
    }
  }

  static void assemble(nh_solver* s, const StagePlan& S) {
    const auto& g = s->grid;
    if (s->one_d) {
      hipLaunchKernelGGL((nh::k_assemble1d<T>), dim3(nblocks(s->ncorn)),
                         dim3(nh::kBlock), 0, s->stream, g.nx, (T)g.dx,
                         P(S.hs_cur), P(S.qa), P(s->H), P(S.wst), s->dt,
                         P(s->cW), P(s->cdiag), P(s->cE), P(s->crhs),
                         bc_mask(s),
                         s->dstats ? &s->dstats->nondom_run : nullptr);
    } else {
      auto a = Args<T>::assemble(s, S);
      hipLaunchKernelGGL((nh::k_assemble2d<T>), dim3(a.nblocks()),
                         dim3(nh::kBlock), 0, s->stream, a);
      if (s->par.solve_norm && s->rhs_max)  // the scale of the residual
        hipLaunchKernelGGL((nh::k_absmax<T>), dim3(1), dim3(nh::kBlock), 0,
                           s->stream, (long)s->ncorn, P(s->crhs),
                           s->rhs_max);
    }
  }

  // nsw <= kSweepS relaxation sweeps starting at sweep index k0 from buffer
  // iin into iout; with check the convergence measure of the input iterate
  // goes to s->part per tile and the input iterate is saved to isave
  // with reduce_seq > 0 the launch also publishes the measure of the
  // preceding check launch under that sequence number
  static void sweeps(nh_solver* s, const SysView& V, bool check, int k0,
                     int nsw, int iin, int iout, int isave,
                     long long reduce_seq = 0) {
    auto a = Args<T>::sweep(s, V);
    nh::SweepLaunch L{iin,        iout, isave, k0, nsw, check ? 1 : 0,
                      reduce_seq > 0 ? 1 : 0, s->E_dev, &s->slot_dev->seq,
                      reduce_seq};
    const dim3 grid(a.nblocks() + (reduce_seq > 0 ? 1 : 0));
    const size_t lds = sweep_lds_bytes(s->tbx, s->tby);
    if (s->sweep_m == nh::kSweepMBig)
      hipLaunchKernelGGL((nh::k_sweep_tb<T, nh::kSweepB, nh::kSweepS,
                                           nh::kSweepMBig>),
                         grid, dim3(nh::kSweepB), lds, s->stream, a, L);
    else
      hipLaunchKernelGGL((nh::k_sweep_tb<T, nh::kSweepB, nh::kSweepS,
                                           nh::kSweepM>),
                         grid, dim3(nh::kSweepB), lds, s->stream, a, L);
  }

  static void thomas(nh_solver* s, void* pout) {
    if (s->par.periodic & 1)  // cyclic system of the nx distinct corners
      hipLaunchKernelGGL((nh::k_thomas_cyclic<T>), dim3(1), dim3(64), 0,
                         s->stream, (int)s->grid.nx, P(s->cW), P(s->cdiag),
                         P(s->cE), P(s->crhs), (double*)pout, s->thomas_bb,
                         s->thomas_z, s->thomas_cp, s->thomas_dp, s->flags);
    else
      hipLaunchKernelGGL((nh::k_thomas<T>), dim3(1), dim3(64), 0, s->stream,
                         (int)s->ncorn, P(s->cW), P(s->cdiag), P(s->cE),
                         P(s->crhs), (double*)pout, s->thomas_cp,
                         s->thomas_dp, s->flags);
  }

  static void correct(nh_solver* s, const StagePlan& S, const void* p) {
    auto a = Args<T>::correct(s, S, p);
    const unsigned nb = a.nblocks(s->one_d);
    if (s->one_d) {
      if (S.combine)
        hipLaunchKernelGGL((nh::k_correct<T, true, true>), dim3(nb),
                           dim3(nh::kBlock), 0, s->stream, a);
      else
        hipLaunchKernelGGL((nh::k_correct<T, true, false>), dim3(nb),
                           dim3(nh::kBlock), 0, s->stream, a);
    } else {
      if (S.combine)
        hipLaunchKernelGGL((nh::k_correct<T, false, true>), dim3(nb),
                           dim3(nh::kBlock), 0, s->stream, a);
      else
        hipLaunchKernelGGL((nh::k_correct<T, false, false>), dim3(nb),
                           dim3(nh::kBlock), 0, s->stream, a);
    }
  }

  static void lambda(nh_solver* s) {
    auto a = Args<T>::lambda(s);
    if (s->one_d)
      hipLaunchKernelGGL((nh::k_lambda<T, true>), dim3(a.nblocks()),
                         dim3(nh::kBlock), 0, s->stream, a);
    else
      hipLaunchKernelGGL((nh::k_lambda<T, false>), dim3(a.nblocks()),
                         dim3(nh::kBlock), 0, s->stream, a);
  }
};

// Spin until the device has released sequence number `want` into mapped host
// memory; the stream is polled now and then so that a failed or drained
// stream ends the wait with an error instead of a hang.
nh_status wait_seq(hipStream_t stream, long long* seq_host, long long want) {
  long spins = 0;
  while (__atomic_load_n(seq_host, __ATOMIC_ACQUIRE) != want) {
    if ((++spins & 1023) == 0) {
      hipError_t q = hipStreamQuery(stream);
      if (q != hipSuccess && q != hipErrorNotReady)
        return fail(NH_EDEVICE, std::string("stream error while waiting: ") +
                                    hipGetErrorString(q));
      if (q == hipSuccess && __atomic_load_n(seq_host, __ATOMIC_ACQUIRE) != want)
        return fail(NH_EDEVICE, "convergence measure was not published");
    }
  }
  return NH_OK;
}

// the measure of the solver's check number s->seq (the device keeps running
// the launches queued behind it)
nh_status wait_measure(nh_solver* s, double* E) {
  if (!s->slot) {
    // no mapped host memory (nh_run_noalloc): copy the published slot back
    // once the stream has reached it
    HostSlot hs{};
    HIP_TRY(hipMemcpyAsync(&hs, s->slot_dev, sizeof(hs),
                           hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (hs.seq != s->seq)
      return fail(NH_EDEVICE, "convergence measure was not published");
    *E = hs.E[0];
    return NH_OK;
  }
  nh_status st = wait_seq(s->stream, &s->slot->seq, s->seq);
  if (st != NH_OK) return st;
  *E = s->slot->E[0];
  return NH_OK;
}

// Relaxation solve of the system V from its iterate in buffer `pcur` (which
// receives the buffer of the result): cycles of check_every sweeps, the
// measure of eq. (32) taken at each cycle start, stop below `tol`.
template <typename T>
nh_status solve2d(nh_solver* s, const SysView& V, int& pcur, double tol,
                  int32_t* sweeps, double* measure) {
  const int ce = s->par.check_every > 0 ? s->par.check_every : 1;
  const int kmax = s->par.solve_max_iter;
  const int S = nh::kSweepS;
  const int kAhead = 1;  // launches queued before waiting for a measure
  int k = 0;             // sweep index of the iterate in buffer `cur`
  int cur = pcur;
  double E = 0.0;
  nh_status st = NH_OK;
  int launches = 0, nsweeps_done = 0;
  for (;;) {
    const int save = (cur + 2) % 3, out = (cur + 1) % 3;
    const int kc = k;
    int nsw = k >= kmax ? 0 : std::min(std::min(S, ce), kmax - k);
    Launch<T>::sweeps(s, V, true, k, nsw, cur, out, save);
    ++s->seq;
    launches += 1;
    if (nsw > 0) {
      cur = out;                 // ping-pong between cur and (save's peer)
      k += nsw;
      nsweeps_done += nsw;
    }
    int other = 3 - cur - save;  // the buffer that is neither cur nor save
    // queue the rest of the cycle, the first kAhead launches before waiting;
    // the first of them also publishes the check's measure
    int queued = 0;
    long long pending = s->seq;
    auto queue_until = [&](int limit) {
      while (k % ce != 0 && k < kmax && queued < limit) {
        int n2 = std::min(std::min(S, ce - k % ce), kmax - k);
        Launch<T>::sweeps(s, V, false, k, n2, cur, other, other, pending);
        pending = 0;
        std::swap(cur, other);
        k += n2;
        nsweeps_done += n2;
        ++queued;
        ++launches;
      }
    };
    if (nsw > 0) queue_until(kAhead);
    if (pending)  // no launch follows the check in this cycle
      hipLaunchKernelGGL(nh::k_reduce_measure, dim3(1), dim3(nh::kBlock), 0,
                         s->stream, (const double* const*)s->part_list,
                         (const int*)s->ntiles_list, 1, s->E_dev,
                         &s->slot_dev->seq, s->seq,
                         (const double*)(s->par.solve_norm ? s->rhs_max
                                                           : nullptr));
    nh_status ws = wait_measure(s, &E);
    if (ws != NH_OK) return ws;
    if (E < tol || kc >= kmax) {
      if (!(E < tol)) st = NH_ENOCONV;
      pcur = save;               // p^kc, saved by the check launch
      k = kc;
      break;
    }
    // the rest of the cycle: back-to-back sweep launches (timed as such)
    int before = queued;
    long pm = (k % ce != 0 && k < kmax) ? s->prof.open(s->stream, 4) : -1;
    queue_until(1 << 30);
    s->prof.close(s->stream, pm, queued - before,
                  (double)(queued - before) * nh::kSweepS * s->ncorn);
    (void)nsweeps_done;
  }
  s->solve_launches_last = launches;
  *sweeps = k;
  *measure = E;
  return st;
}

// The kernel instance of the one-launch solve: 1024-thread workgroups,
// blocks of 8 sweeps, 3 points per thread (measured on 513^2 corners: per
// sweep the blocks of 15 sweeps with 8 points per thread in 512-thread
// workgroups took 1.3x as long, the longer blocks saving less exchange time
// than their larger rings and lower occupancy cost)
constexpr int kPersistB = 1024, kPersistS = 8, kPersistM = 3;

template <typename T>
const void* persist_kernel() {
  return (const void*)&nh::k_solve_persist<T, kPersistB, kPersistS,
                                           kPersistM>;
}

// The solve of the system V in one cooperative launch (k_solve_persist) from
// its iterate in buffer `pcur`, which receives the buffer of the result.  The
// host does not wait: the sweep count and the measure go to the device
// statistics, a capped solve to their count of such solves.
// polls before a wait between workgroups gives up (negative: at once)
long long wait_bound(int32_t wait_polls) {
  return wait_polls == 0 ? (1LL << 21) : (long long)wait_polls;
}

template <typename T>
nh_status solve_persist(nh_solver* s, const SysView& V, int& pcur, double tol,
                        int stage) {
  nh::SweepArgs<T> a = Args<T>::sweep(s, V);
  a.BX = s->ptbx;
  a.BY = s->ptby;
  a.ntx = s->pntx;
  a.ntiles = s->pntx * s->pnty;
  a.part = nullptr;
  const int ce = s->par.check_every > 0 ? s->par.check_every : 1;
  const long pk = s->prof.open(s->stream, 5);
  nh::PersistLaunch L{pcur, (pcur + 1) % 3, s->par.solve_max_iter, ce,
                      stage, pk >= 0 ? 1 : 0, tol};
  // a wait gives up after ~2^21 polls (seconds; a block of sweeps takes
  // microseconds), or at once for a negative wait_polls
  nh::PersistSync Y{s->p_xch, s->p_xch + 2 * s->ncorn, s->p_bar,
                    s->p_slots, s->flags, s->dstats,
                    wait_bound(s->par.wait_polls)};
  void* args[] = {&a, &L, &Y};
  // solve_path 2 asks the runtime to guarantee that every workgroup is
  // resident (a cooperative launch, ~20 us more per solve on the device's
  // timeline); otherwise a plain launch of no more workgroups than the
  // device holds at once: with the stream's earlier work complete they are
  // all resident, and if other work on the device delays some, the waits
  // of the others are bounded and the run reports NH_EDEVICE
  hipError_t e =
      s->par.solve_path == 2
          ? hipLaunchCooperativeKernel(persist_kernel<T>(), dim3(a.ntiles),
                                       dim3(kPersistB), args,
                                       (unsigned)s->plds, s->stream)
          : hipLaunchKernel(persist_kernel<T>(), dim3(a.ntiles),
                            dim3(kPersistB), args, (unsigned)s->plds,
                            s->stream);
  s->prof.close(s->stream, pk, 1);
  if (e != hipSuccess)
    return fail(NH_EDEVICE, std::string("one-launch solve: ") +
                                hipGetErrorString(e));
  pcur = L.iout;
  s->solve_launches_last = 1;
  return NH_OK;
}

template <typename T>
nh_status stage(nh_solver* s, int idx, int32_t* sweeps, double* measure) {
  StagePlan S = stage_plan(s, idx);
  s->hs_cur = S.hs_cur;
  long pm = s->prof.open(s->stream, 0);
  Launch<T>::fv(s, S);
  if (s->par.w_advection) {
    // energy-consistent form: w carried by the stage input's flow; the rest
    // of the stage (breaking, assembly, correction) reads the carried w
    Launch<T>::advect_w(s, S, s->wadv);
    S.w_in = s->wadv;
    if (!s->par.breaking_on) S.wst = s->wadv;
  }
  s->prof.close(s->stream, pm, s->par.w_advection ? 2 : 1);
  pm = s->prof.open(s->stream, 1);
  if (s->par.breaking_on) Launch<T>::breaking(s, S);
  if (s->par.nh_on) Launch<T>::assemble(s, S);
  s->prof.close(s->stream, pm,
                (s->par.breaking_on ? 2 : 0) + (s->par.nh_on ? 1 : 0));
  nh_status st = NH_OK;
  *sweeps = 0;
  *measure = 0.0;
  const void* p = nullptr;
  if (s->par.nh_on) {
    pm = s->prof.open(s->stream, 2);
    if (s->one_d) {
      Launch<T>::thomas(s, s->pcur_ptr());
      s->solve_launches_last = 1;
    } else if (s->persist) {
      st = solve_persist<T>(s, forward_system(s), s->pcur, s->par.solve_tol,
                            idx);
      if (st != NH_OK) return st;
    } else {
      st = solve2d<T>(s, forward_system(s), s->pcur, s->par.solve_tol, sweeps,
                      measure);
      if (st != NH_OK && st != NH_ENOCONV) return st;
    }
    s->prof.close(s->stream, pm, s->solve_launches_last);
    p = s->pcur_ptr();
    if (s->tape_p[idx])
      hipMemcpyAsync(s->tape_p[idx], p, s->ncorn * sizeof(double),
                     hipMemcpyDeviceToDevice, s->stream);
  }
  pm = s->prof.open(s->stream, 3);
  Launch<T>::correct(s, S, p);
  if (S.combine && s->relax_on && p)
    hipLaunchKernelGGL((nh::k_relax_p<T>), dim3(nblocks(s->ncorn)),
                       dim3(nh::kBlock), 0, s->stream, (int)s->ncorn,
                       (double*)p, (const T*)s->rm_k, s->rt_p);
  s->prof.close(s->stream, pm, 1);
  return st;
}

// Host view of the device-side statistics (t, dt, flags, clamped mass),
// refreshed at synchronisation points.
nh_status sync_stats(nh_solver* s) {
  // the water volume of the state (per-workgroup sums, then one workgroup)
  const unsigned nbc = nblocks(s->ncell);
  if (s->fp32)
    hipLaunchKernelGGL((nh::k_depth_sums<float>), dim3(nbc), dim3(nh::kBlock),
                       0, s->stream, s->ncell, (const float*)s->h,
                       (const float*)s->H, s->lampart);
  else
    hipLaunchKernelGGL((nh::k_depth_sums<double>), dim3(nbc),
                       dim3(nh::kBlock), 0, s->stream, s->ncell,
                       (const double*)s->h, (const double*)s->H, s->lampart);
  hipLaunchKernelGGL(nh::k_sum_parts, dim3(1), dim3(nh::kBlock), 0, s->stream,
                     (int)nbc, (const double*)s->lampart, s->dstats);
  nh::DevStats ds{};
  int flags = 0;
  double dt_next = 0.0, clamped = 0.0;
  HIP_TRY(hipMemcpyAsync(&ds, s->dstats, sizeof(ds), hipMemcpyDeviceToHost,
                         s->stream));
  HIP_TRY(hipMemcpyAsync(&dt_next, s->dt, sizeof(double),
                         hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipMemcpyAsync(&flags, s->flags, sizeof(int), hipMemcpyDeviceToHost,
                         s->stream));
  HIP_TRY(hipMemcpyAsync(&clamped, s->clamped, sizeof(double),
                         hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->prof.flush();
  s->st.t = ds.t;
  s->st.dt_last = ds.dt_last;
  s->st.step = ds.step;
  s->st.dt_next = dt_next;
  s->st.clamped_mass = clamped;
  s->st.mass = ds.depth_sum * s->grid.dx * (s->one_d ? 1.0 : s->grid.dy);
  s->st.nondominant = ds.nondom_last;
  bool capped = false;
  if (s->persist && s->par.nh_on) {
    s->st.sweeps[0] = ds.sweeps[0];
    s->st.sweeps[1] = ds.sweeps[1];
    s->st.measure = ds.measure;
    s->st.sweeps_total = ds.sweeps_total;
    s->st.solves_total = ds.solves_total;
    capped = ds.noconv > s->noconv_seen;
    s->noconv_seen = ds.noconv;
  }
  nh_status st = NH_OK;
  if (flags & 1) st = fail(NH_ENONFINITE, "non-finite value in the state");
  if (flags & 2 && st == NH_OK)
    st = fail(NH_EDEVICE, "singular tridiagonal system");
  if (flags & 4 && st == NH_OK)
    st = fail(NH_ESTATE, "no wet cell: the CFL time step is undefined");
  if (flags & nh::kFlagWaitBound && st == NH_OK)
    st = fail(NH_EDEVICE,
              "one-launch solve: a wait between workgroups reached its bound "
              "(other work on the device kept some workgroups out; "
              "solve_path 2 launches cooperatively)");
  if (st != NH_OK) {
    s->st.last_status = st;
    s->have_state = false;
    return st;
  }
  if (capped) {
    // the state stays valid
    s->st.last_status = NH_ENOCONV;
    return fail(NH_ENOCONV, "pressure solve reached solve_max_iter");
  }
  return NH_OK;
}

// One step, queued on the stream.  The host waits only for the solver's
// convergence decisions; dt, t and the status stay on the device until the
// next sync_stats.
template <typename T>
nh_status step_impl(nh_solver* s) {
  int32_t sw1 = 0, sw2 = 0;
  double m1 = 0.0, m2 = 0.0;
  // stage 1: U^n -> U^(1)  (h* of stage 1 in hs)
  nh_status st = stage<T>(s, 0, &sw1, &m1);
  if (st != NH_OK && st != NH_ENOCONV) return st;
  // stage 2: U^(1) -> U^(2), averaged into U^n
  nh_status st2 = stage<T>(s, 1, &sw2, &m2);
  if (st2 != NH_OK && st2 != NH_ENOCONV) return st2;
  if (st == NH_OK) st = st2;
  nh::FinalizeArgs fa = finalize_args(s, true);
  hipLaunchKernelGGL(nh::k_finalize_dt, dim3(1), dim3(nh::kBlock), 0,
                     s->stream, fa);
  if (!(s->persist && s->par.nh_on)) {
    // one-launch solves count on the device (sync_stats)
    s->st.sweeps[0] = sw1;
    s->st.sweeps[1] = sw2;
    s->st.sweeps_total += sw1 + sw2;
    s->st.solves_total += s->par.nh_on ? 2 : 0;
    s->st.measure = m2;
  }
  if (st == NH_ENOCONV) fail(st, "pressure solve reached solve_max_iter");
  s->st.last_status = st;
  return st;
}

nh_status check_params(const nh_grid* g, const nh_params* p) {
  if (!g || !p) return fail(NH_EINVAL, "null grid or params");
  if (g->nx < 2 || g->ny < 1)
    return fail(NH_EINVAL, "need nx >= 2 and ny == 1 or ny >= 2");
  if ((long)g->nx * (long)(g->ny + 1) > (1L << 30))
    return fail(NH_EINVAL, "grid too large");
  if (!(g->dx > 0) || (g->ny > 1 && !(g->dy > 0)))
    return fail(NH_EINVAL, "dx, dy must be > 0");
  if (!(p->g > 0) || !(p->cfl > 0) || p->cfl > 1.0)
    return fail(NH_EINVAL, "need g > 0 and 0 < cfl <= 1");
  if (!(p->delta > 0) || !(p->dry_eps >= 0))
    return fail(NH_EINVAL, "need delta > 0 and dry_eps >= 0");
  if (!(p->manning >= 0) || !std::isfinite(p->manning))
    return fail(NH_EINVAL, "need a finite manning >= 0");
  if (p->open_sides < 0 || p->open_sides > 15)
    return fail(NH_EINVAL, "open_sides is a mask of 4 bits");
  if (p->periodic < 0 || p->periodic > 3)
    return fail(NH_EINVAL, "periodic is a mask of 2 bits");
  if (p->w_advection != 0 && p->w_advection != 1)
    return fail(NH_EINVAL, "w_advection must be 0 or 1");
  if (((p->periodic & 1) && (p->open_sides & 3)) ||
      (g->ny > 1 && (p->periodic & 2) && (p->open_sides & 12)))
    return fail(NH_EINVAL, "a periodic direction has no open side");
  if (p->precision != NH_FP64 && p->precision != NH_FP32)
    return fail(NH_EINVAL, "precision must be NH_FP64 or NH_FP32");
  if (p->solve_path < 0 || p->solve_path > 2)
    return fail(NH_EINVAL, "solve_path must be 0, 1 or 2");
  if (p->solve_norm != 0 && p->solve_norm != 1)
    return fail(NH_EINVAL, "solve_norm must be 0 or 1");
  if (p->nh_on && g->ny > 1) {
    if (p->solve_max_iter < 0) return fail(NH_EINVAL, "solve_max_iter < 0");
    int nom = (p->omega_schedule && p->n_omega > 0) ? p->n_omega : 1;
    int ce = p->check_every > 0 ? p->check_every : 1;
    if (ce % nom != 0)
      return fail(NH_EINVAL, "check_every must be a multiple of n_omega");
    if (p->omega_schedule && p->n_omega > 0)
      for (int i = 0; i < p->n_omega; ++i)
        if (!(p->omega_schedule[i] > 0) || !std::isfinite(p->omega_schedule[i]))
          return fail(NH_EINVAL, "relaxation factors must be finite and > 0");
  }
  if (p->fixed_dt && !(p->dt > 0)) return fail(NH_EINVAL, "fixed dt must be > 0");
  return NH_OK;
}

// sweep tiles of a solver's grid
nh_status choose_sweep_tiles(nh_solver* s) {
  // sweep tiles: 24 x 24 corners with a halo of kSweepS and 2 region points
  // per thread (measured best of the tile/halo/workgroup shapes tried on
  // gfx950 for 513^2 corners); FP32-bulk grids of more than 1024 such tiles
  // take 32 x 32 tiles with 3 points per thread (fewer halo re-reads; in
  // FP64 the 3-point kernel needs more than 64 registers and loses half its
  // occupancy).  The region must fit kSweepB * sweep_m points (checked here,
  // assumed by the kernel).
  s->tbx = 24;
  s->tby = 24;
  s->sweep_m = nh::kSweepM;
  if (!s->one_d && s->fp32 &&
      (long)((s->grid.nx + 24) / 24) * ((s->grid.ny + 24) / 24) > 1024) {
    s->tbx = 32;
    s->tby = 32;
    s->sweep_m = nh::kSweepMBig;
  }
  if ((s->tbx + 2 * nh::kSweepS) * (s->tby + 2 * nh::kSweepS) >
      nh::kSweepB * s->sweep_m) {
    return fail(NH_EINVAL, "sweep tile does not fit the workgroup");
  }
  s->ntx = (s->grid.nx + 1 + s->tbx - 1) / s->tbx;
  s->nty = s->one_d ? 1 : (s->grid.ny + 1 + s->tby - 1) / s->tby;
  return NH_OK;
}

// Tiles of the one-launch solve: a tile's region (its corners and those
// within kPersistS of them) must fit the workgroup's threads (a column
// segment of kPersistM points each) and its LDS (two padded FP64 planes),
// and the tiles -- counted over the distinct corners of a periodic line --
// may not outnumber the workgroups of the kernel that the device holds at
// once; of those tilings the smallest region wins.  Leaves s->persist false
// when none fits (NH_EINVAL if solve_path demands the one launch).
template <typename T>
nh_status choose_persist_tiles_t(nh_solver* s) {
  const int B = kPersistB, S = kPersistS, M = kPersistM;
  const int ncx = s->grid.nx + 1, ncy = s->grid.ny + 1;
  const int nlx = (s->par.periodic & 1) ? ncx - 1 : ncx;
  const int nly = (s->par.periodic & 2) ? ncy - 1 : ncy;
  int coop = 0, cus = 0, lds_dev = 0;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch,
                            s->device) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                            s->device) != hipSuccess ||
      hipDeviceGetAttribute(&lds_dev,
                            hipDeviceAttributeMaxSharedMemoryPerBlock,
                            s->device) != hipSuccess) {
    (void)hipGetLastError();
    coop = 0;
  }
  if ((long)ncx * ncy >= (1L << 26)) coop = 0;  // corner index << 5 in int
  if (s->nom > nh::kPersistOmega) coop = 0;     // the schedule lives in LDS
  const void* kern = persist_kernel<T>();
  // LDS of the widest region (rows of B threads)
  const size_t lds_cap =
      std::min<size_t>((size_t)lds_dev, nh::persist_lds_bytes(B, M, B));
  if (coop && lds_cap > 65536 &&
      hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lds_cap) != hipSuccess) {
    (void)hipGetLastError();
    coop = 0;
  }
  int per_cu = 0;
  if (coop && hipOccupancyMaxActiveBlocksPerMultiprocessor(
                  &per_cu, kern, B, lds_cap) != hipSuccess) {
    (void)hipGetLastError();
    per_cu = 0;
  }
  const long cap = (long)per_cu * cus;
  long best_area = 0, nt_b = 0;
  int bx_b = 0, by_b = 0;
  for (int bx = 1; coop && bx + 2 * S <= B; ++bx)
    for (int by = 1; by + 2 * S <= B; ++by) {
      const long rw = bx + 2 * S, rh = by + 2 * S;
      if (rw * ((rh + M - 1) / M) > B) break;
      if ((size_t)nh::persist_lds_bytes(B, M, (int)rw) > lds_cap) break;
      const long area = rw * rh;
      const long nt = (long)((nlx + bx - 1) / bx) * ((nly + by - 1) / by);
      if (nt > cap) continue;
      if (best_area == 0 || area < best_area ||
          (area == best_area && nt < nt_b)) {
        best_area = area;
        bx_b = bx;
        by_b = by;
        nt_b = nt;
      }
    }
  if (best_area == 0) {
    if (s->par.solve_path == 2)
      return fail(NH_EINVAL,
                  "solve_path 2: the grid's tiles do not fit the co-resident "
                  "workgroups of the device");
    return NH_OK;
  }
  s->ptbx = bx_b;
  s->ptby = by_b;
  s->pntx = (nlx + bx_b - 1) / bx_b;
  s->pnty = (nly + by_b - 1) / by_b;
  s->plds = nh::persist_lds_bytes(B, M, bx_b + 2 * S);
  s->persist = true;
  return NH_OK;
}

nh_status choose_persist_tiles(nh_solver* s) {
  s->persist = false;
  if (s->one_d || !s->par.nh_on || s->par.solve_path == 1) return NH_OK;
  return s->fp32 ? choose_persist_tiles_t<float>(s)
                 : choose_persist_tiles_t<double>(s);
}

// with U^n (h, q1, q2, w) in place on the device: p from the host array
// (device array with p_on_device), or 0; statistics reset, dt from the CFL
// condition (or the fixed dt)
nh_status adopt_state(nh_solver* s, const double* p, bool p_on_device = false) {
  s->pcur = 0;
  if (p) {
    HIP_TRY(hipMemcpyAsync(s->pa, p, s->ncorn * sizeof(double),
                           p_on_device ? hipMemcpyDeviceToDevice
                                       : hipMemcpyHostToDevice,
                           s->stream));
  } else {
    HIP_TRY(hipMemsetAsync(s->pa, 0, s->ncorn * sizeof(double), s->stream));
  }
  HIP_TRY(hipMemsetAsync(s->flags, 0, sizeof(int), s->stream));
  HIP_TRY(hipMemsetAsync(s->clamped, 0, sizeof(double), s->stream));
  HIP_TRY(hipMemsetAsync(s->dstats, 0, sizeof(nh::DevStats), s->stream));
  s->noconv_seen = 0;
  if (s->persist) {
    // tags from 0 again (also after a failed solve)
    HIP_TRY(hipMemsetAsync(s->p_xch, 0,
                           4 * (size_t)s->ncorn * sizeof(unsigned long long),
                           s->stream));
    HIP_TRY(hipMemsetAsync(s->p_bar, 0, 2 * sizeof(unsigned), s->stream));
    HIP_TRY(hipMemsetAsync(
        s->p_slots, 0,
        4 * (size_t)s->pntx * s->pnty * sizeof(unsigned long long),
        s->stream));
  }
  double dt0 = 0.0;
  if (s->par.fixed_dt) {
    dt0 = s->par.dt;
    HIP_TRY(hipMemcpyAsync(s->dt, &dt0, sizeof(double), hipMemcpyHostToDevice,
                           s->stream));
  } else {
    if (s->fp32)
      Launch<float>::lambda(s);
    else
      Launch<double>::lambda(s);
    nh::FinalizeArgs fa = finalize_args(s, false);
    hipLaunchKernelGGL(nh::k_finalize_dt, dim3(1), dim3(nh::kBlock), 0,
                       s->stream, fa);
    HIP_TRY(hipMemcpyAsync(&dt0, s->dt, sizeof(double), hipMemcpyDeviceToHost,
                           s->stream));
  }
  int flags = 0;
  HIP_TRY(hipMemcpyAsync(&flags, s->flags, sizeof(int), hipMemcpyDeviceToHost,
                         s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  HIP_TRY(hipMemsetAsync(s->flags, 0, sizeof(int), s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  std::memset(&s->st, 0, sizeof(s->st));
  s->st.dt_next = dt0;
  if (flags & 4) {
    s->have_state = false;
    return fail(NH_ESTATE, "no wet cell: the CFL time step is undefined");
  }
  s->have_state = true;
  return NH_OK;
}

// a view handed to nh_bind_device_buffers: device memory of the solver's
// device, aligned to the element size, with n elements inside its allocation
nh_status check_view(const nh_solver* s, const void* p, long n) {
  if (reinterpret_cast<uintptr_t>(p) % s->esize != 0)
    return fail(NH_EINVAL, "device view not aligned to the element size");
  hipPointerAttribute_t at{};
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return fail(NH_EINVAL, "view is not device memory");
  }
  if (at.type != hipMemoryTypeDevice || at.device != s->device)
    return fail(NH_EINVAL, "view is not device memory of the solver's device");
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, const_cast<void*>(p)) !=
      hipSuccess) {
    (void)hipGetLastError();
    return fail(NH_EINVAL, "view is not inside a device allocation");
  }
  const char* b = static_cast<const char*>(base);
  const char* q = static_cast<const char*>(p);
  if (q < b || q + (size_t)n * s->esize > b + size)
    return fail(NH_EINVAL, "view extends past the end of its allocation");
  return NH_OK;
}

// frees a buffer the solver allocated itself (borrowed ones are left alone)
void release_own(nh_solver* s, void* p) {
  auto it = std::find(s->allocs.begin(), s->allocs.end(), p);
  if (it != s->allocs.end()) {
    (void)hipFree(p);
    s->allocs.erase(it);
  }
}

// H (nullable): `a` holds stored depth values, checked as depths
template <typename T>
void check_values(nh_solver* s, const void* a, long n, int nf, int neg,
                  const void* H = nullptr) {
  hipLaunchKernelGGL((nh::k_check_values<T>), dim3(nblocks(n)),
                     dim3(nh::kBlock), 0, s->stream, n,
                     static_cast<const T*>(a), nf, neg, s->flags,
                     static_cast<const T*>(H));
}

}  // namespace

extern "C" {

const char* nh_last_error(void) { return g_err.c_str(); }

const char* nh_version(void) { return "nhswe-gfx950 0.1"; }

nh_status nh_create(const nh_grid* grid, const nh_params* params,
                    void* hip_stream, nh_solver** out) {
  if (!out) return fail(NH_EINVAL, "null output pointer");
  *out = nullptr;
  nh_status st = check_params(grid, params);
  if (st != NH_OK) return st;
  nh_solver* s = new nh_solver();
  s->grid = *grid;
  s->par = *params;
  if (params->omega_schedule && params->n_omega > 0)
    s->omega.assign(params->omega_schedule,
                    params->omega_schedule + params->n_omega);
  else
    s->omega.assign(1, 1.0);
  s->nom = (int)s->omega.size();
  s->par.omega_schedule = nullptr;
  s->one_d = grid->ny == 1;
  s->fp32 = params->precision == NH_FP32;
  s->esize = s->fp32 ? 4 : 8;
  if (hip_stream) {
    s->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreate(&s->stream) != hipSuccess) {
      delete s;
      return fail(NH_EDEVICE, "hipStreamCreate failed");
    }
    s->own_stream = true;
  }
  if (hipGetDevice(&s->device) != hipSuccess) {
    if (s->own_stream) hipStreamDestroy(s->stream);
    delete s;
    return fail(NH_EDEVICE, "hipGetDevice failed");
  }
  s->ncell = (long)grid->nx * grid->ny;
  s->ncorn = (long)(grid->nx + 1) * (s->one_d ? 1 : grid->ny + 1);
  size_t cb = s->ncell * s->esize, kb = s->ncorn * s->esize;
  void** cells[] = {&s->H,   &s->h,   &s->q1,  &s->q2,  &s->hs,  &s->q1s,
                    &s->q2s, &s->q1b, &s->q2b, &s->rw,  &s->h1,  &s->q11,
                    &s->q21};
  void** corners[] = {&s->w,  &s->ws, &s->w1, &s->wadv, &s->cdiag,
                      &s->cE, &s->cW, &s->cN, &s->cS, &s->crhs};
  for (auto c : cells)
    if ((st = dalloc(s, c, cb)) != NH_OK) { nh_destroy(s); return st; }
  for (auto c : corners)
    if ((st = dalloc(s, c, kb)) != NH_OK) { nh_destroy(s); return st; }
  for (auto c : {&s->pa, &s->pb, &s->pc})
    if ((st = dalloc(s, c, s->ncorn * sizeof(double))) != NH_OK) {
      nh_destroy(s);
      return st;
    }
  long nstage = s->ncell > s->ncorn ? s->ncell : s->ncorn;
  if ((st = dalloc(s, &s->stage_buf, nstage * sizeof(double))) != NH_OK ||
      (st = dalloc(s, (void**)&s->thomas_cp, s->ncorn * sizeof(double))) != NH_OK ||
      (st = dalloc(s, (void**)&s->thomas_dp, s->ncorn * sizeof(double))) != NH_OK ||
      (st = dalloc(s, (void**)&s->thomas_bb, s->ncorn * sizeof(double))) != NH_OK ||
      (st = dalloc(s, (void**)&s->thomas_z, s->ncorn * sizeof(double))) != NH_OK ||
      (st = dalloc(s, (void**)&s->dt, sizeof(double))) != NH_OK ||
      (st = dalloc(s, (void**)&s->lampart,
                   nblocks(std::max(s->ncell, s->ncorn)) * sizeof(double))) !=
          NH_OK ||

      (st = dalloc(s, (void**)&s->omega_dev,
                   s->omega.size() * sizeof(double))) != NH_OK ||
      (st = dalloc(s, (void**)&s->clamped, sizeof(double))) != NH_OK ||
      (st = dalloc(s, (void**)&s->flags, sizeof(int))) != NH_OK) {
    nh_destroy(s);
    return st;
  }
  if (hipMemcpyAsync(s->omega_dev, s->omega.data(),
                     s->omega.size() * sizeof(double), hipMemcpyHostToDevice,
                     s->stream) != hipSuccess) {
    nh_destroy(s);
    return fail(NH_EDEVICE, "copy of the relaxation schedule failed");
  }
  if ((st = choose_sweep_tiles(s)) != NH_OK ||
      (st = choose_persist_tiles(s)) != NH_OK) {
    nh_destroy(s);
    return st;
  }
  if (s->par.solve_norm && s->par.nh_on && !s->one_d &&
      dalloc(s, (void**)&s->rhs_max, sizeof(double)) != NH_OK) {
    nh_destroy(s);
    return fail(NH_ENOMEM, "allocation of the residual scale failed");
  }
  if (s->persist) {
    const size_t nt = (size_t)s->pntx * s->pnty;
    const size_t xb = 4 * (size_t)s->ncorn * sizeof(unsigned long long);
    const size_t sb = 4 * nt * sizeof(unsigned long long);
    if (dalloc(s, (void**)&s->p_xch, xb) != NH_OK ||
        dalloc(s, (void**)&s->p_bar, 2 * sizeof(unsigned)) != NH_OK ||
        dalloc(s, (void**)&s->p_slots, sb) != NH_OK ||
        hipMemset(s->p_xch, 0, xb) != hipSuccess ||
        hipMemset(s->p_bar, 0, 2 * sizeof(unsigned)) != hipSuccess ||
        hipMemset(s->p_slots, 0, sb) != hipSuccess) {
      nh_destroy(s);
      return fail(NH_ENOMEM, "allocation of the one-launch solve's counters "
                             "failed");
    }
  }
  if (dalloc(s, (void**)&s->dstats, sizeof(nh::DevStats)) != NH_OK ||
      hipHostMalloc((void**)&s->slot, sizeof(HostSlot),
                    hipHostMallocMapped | hipHostMallocCoherent) !=
          hipSuccess ||
      hipHostGetDevicePointer((void**)&s->slot_dev, s->slot, 0) !=
          hipSuccess) {
    nh_destroy(s);
    return fail(NH_ENOMEM, "allocation of the statistics buffers failed");
  }
  s->slot->E[0] = 0.0;
  s->slot->seq = 0;
  s->seq = 0;
  s->E_dev = &s->slot_dev->E[0];
  int ntiles_h = s->ntx * s->nty;
  if (dalloc(s, (void**)&s->part, s->ntx * s->nty * sizeof(double)) !=
          NH_OK ||
      dalloc(s, (void**)&s->part_list, sizeof(double*)) != NH_OK ||
      dalloc(s, (void**)&s->ntiles_list, sizeof(int)) != NH_OK ||
      hipMemcpy(s->part_list, &s->part, sizeof(double*),
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(s->ntiles_list, &ntiles_h, sizeof(int),
                hipMemcpyHostToDevice) != hipSuccess) {
    nh_destroy(s);
    return fail(NH_ENOMEM, "allocation of the convergence buffers failed");
  }
  if (hipStreamSynchronize(s->stream) != hipSuccess) {
    nh_destroy(s);
    return fail(NH_EDEVICE, "stream synchronisation failed");
  }
  *out = s;
  return NH_OK;
}

nh_status nh_set_bathymetry(nh_solver* s, const double* H) {
  if (!s || !H) return fail(NH_EINVAL, "null argument");
  for (long i = 0; i < s->ncell; ++i)
    if (!std::isfinite(H[i])) return fail(NH_EINVAL, "non-finite bathymetry");
  nh_status st = upload(s, s->H, H, s->ncell);
  if (st == NH_OK) {
    s->have_H = true;
    if (s->fp32) s->H_host.assign(H, H + s->ncell);
  }
  return st;
}

// weights of the generation/absorption zones along one direction of n cells
// (low and high walls of widths Llo, Lhi): the k + 1 cells nearest a wall
// with a zone, k the least natural number with k dx >= L, get
// m = sqrt(max(0, 1 - (d/L)^2)), d the distance to the zone's innermost cell
static void zone_profile(int n, double dx, double Llo, double Lhi,
                         std::vector<double>& m) {
  m.assign(n, 1.0);
  const double L[2] = {Llo, Lhi};
  for (int side = 0; side < 2; ++side) {
    if (!(L[side] > 0.0)) continue;
    long k = (long)std::ceil(L[side] / dx);
    while (k > 0 && (double)(k - 1) * dx >= L[side]) --k;
    for (long r = 0; r <= k; ++r) {
      const long i = side == 0 ? k - r : n - 1 - k + r;
      if (i < 0 || i >= n) continue;
      const double d = (double)r * dx / L[side];
      m[i] *= std::sqrt(std::max(0.0, 1.0 - d * d));
    }
  }
}

nh_status nh_set_relaxation(nh_solver* s, const double* widths,
                            const double* h_t, const double* q1_t,
                            const double* q2_t, const double* w_t,
                            const double* p_t) {
  if (!s || !widths) return fail(NH_EINVAL, "null argument");
  for (int i = 0; i < 4; ++i)
    if (!(widths[i] >= 0.0) || !std::isfinite(widths[i]))
      return fail(NH_EINVAL, "zone widths must be finite and >= 0");
  if (((s->par.periodic & 1) && (widths[0] > 0 || widths[1] > 0)) ||
      (!s->one_d && (s->par.periodic & 2) && (widths[2] > 0 || widths[3] > 0)))
    return fail(NH_EINVAL, "no relaxation zone across a periodic direction");
  const bool on = widths[0] > 0 || widths[1] > 0 ||
                  (!s->one_d && (widths[2] > 0 || widths[3] > 0));
  s->relax_on = false;
  if (!on) return NH_OK;
  if (!h_t && !s->have_H) return fail(NH_ESTATE, "set the bathymetry first");
  const int nx = s->grid.nx, ny = s->one_d ? 1 : s->grid.ny;
  const int ncx = nx + 1, ncy = s->one_d ? 1 : ny + 1;
  std::vector<double> mx, my;
  zone_profile(nx, s->grid.dx, widths[0], widths[1], mx);
  if (s->one_d)
    my.assign(1, 1.0);
  else
    zone_profile(ny, s->grid.dy, widths[2], widths[3], my);
  auto mir = [](int i, int n) {
    return i < 0 ? -1 - i : (i >= n ? 2 * n - 1 - i : i);
  };
  std::vector<double> mc(s->ncell), mk(s->ncorn), th(s->ncell), tq1(s->ncell),
      tq2(s->ncell), tw(s->ncorn), tp(s->ncorn);
  std::vector<double> Hh;
  nh_status st;
  if (!h_t) {  // still water: h* = max(H, 0)
    Hh.resize(s->ncell);
    if ((st = download(s, Hh.data(), s->H, s->ncell)) != NH_OK) return st;
  }
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const long c = (long)j * nx + i;
      mc[c] = mx[i] * my[j];
      th[c] = h_t ? h_t[c] : std::max(Hh[c], 0.0);
      tq1[c] = q1_t ? q1_t[c] : 0.0;
      tq2[c] = q2_t ? q2_t[c] : 0.0;
    }
  for (int l = 0; l < ncy; ++l)
    for (int k = 0; k < ncx; ++k) {
      const long c = (long)l * ncx + k;
      const double ax = 0.5 * (mx[mir(k - 1, nx)] + mx[mir(k, nx)]);
      const double ay =
          s->one_d ? 1.0 : 0.5 * (my[mir(l - 1, ny)] + my[mir(l, ny)]);
      mk[c] = ax * ay;
      tw[c] = w_t ? w_t[c] : 0.0;
      tp[c] = p_t ? p_t[c] : 0.0;
    }
  for (long c = 0; c < s->ncell; ++c)
    if (!std::isfinite(th[c]) || !std::isfinite(tq1[c]) ||
        !std::isfinite(tq2[c]) || th[c] < 0.0)
      return fail(NH_EINVAL, "targets must be finite, with h* >= 0");
  for (long c = 0; c < s->ncorn; ++c)
    if (!std::isfinite(tw[c]) || !std::isfinite(tp[c]))
      return fail(NH_EINVAL, "targets must be finite");
  if (!s->rm_c) {  // first use: the zone arrays, kept for the solver's life
    void** cells[] = {&s->rm_c, &s->rt_h, &s->rt_q1, &s->rt_q2};
    void** corners[] = {&s->rm_k, &s->rt_w};
    for (auto a : cells)
      if ((st = dalloc(s, a, s->ncell * s->esize)) != NH_OK) return st;
    for (auto a : corners)
      if ((st = dalloc(s, a, s->ncorn * s->esize)) != NH_OK) return st;
    if ((st = dalloc(s, (void**)&s->rt_p, s->ncorn * sizeof(double))) !=
        NH_OK)
      return st;
  }
  if ((st = upload(s, s->rm_c, mc.data(), s->ncell)) != NH_OK ||
      (st = upload_depth(s, s->rt_h, th.data(), s->ncell)) != NH_OK ||
      (st = upload(s, s->rt_q1, tq1.data(), s->ncell)) != NH_OK ||
      (st = upload(s, s->rt_q2, tq2.data(), s->ncell)) != NH_OK ||
      (st = upload(s, s->rm_k, mk.data(), s->ncorn)) != NH_OK ||
      (st = upload(s, s->rt_w, tw.data(), s->ncorn)) != NH_OK)
    return st;
  HIP_TRY(hipMemcpyAsync(s->rt_p, tp.data(), s->ncorn * sizeof(double),
                         hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->relax_on = true;
  return NH_OK;
}

nh_status nh_set_state(nh_solver* s, const double* h, const double* hu,
                       const double* hv, const double* w, const double* p) {
  if (!s || !h || !hu) return fail(NH_EINVAL, "null argument");
  if (!s->have_H) return fail(NH_ESTATE, "set the bathymetry first");
  for (long i = 0; i < s->ncell; ++i) {
    if (!std::isfinite(h[i]) || !std::isfinite(hu[i]) ||
        (hv && !s->one_d && !std::isfinite(hv[i])))
      return fail(NH_EINVAL, "non-finite state");
    if (h[i] < 0.0) return fail(NH_ENEGDEPTH, "negative depth");
  }
  nh_status st;
  if ((st = upload_depth(s, s->h, h, s->ncell)) != NH_OK) return st;
  if ((st = upload(s, s->q1, hu, s->ncell)) != NH_OK) return st;
  if (hv && !s->one_d) {
    if ((st = upload(s, s->q2, hv, s->ncell)) != NH_OK) return st;
  } else {
    HIP_TRY(hipMemsetAsync(s->q2, 0, s->ncell * s->esize, s->stream));
  }
  if (w) {
    if ((st = upload(s, s->w, w, s->ncorn)) != NH_OK) return st;
  } else {
    HIP_TRY(hipMemsetAsync(s->w, 0, s->ncorn * s->esize, s->stream));
  }
  return adopt_state(s, p);
}

nh_status nh_bind_device_buffers(nh_solver* s, const nh_device_views* v) {
  if (!s || !v) return fail(NH_EINVAL, "null argument");
  const bool state = v->h || v->hu || v->hv || v->w;
  if (!v->H && !state) return fail(NH_EINVAL, "no view given");
  if (s->one_d && v->hv) return fail(NH_EINVAL, "hv is not used in 1D");
  if (state && (!v->h || !v->hu || (!s->one_d && !v->hv)))
    return fail(NH_EINVAL, "h and hu (and hv in 2D) are bound together");
  if (state && !v->H && !s->have_H)
    return fail(NH_ESTATE, "set or bind the bathymetry first");
  const void* views[5] = {v->H, v->h, v->hu, v->hv, v->w};
  const long counts[5] = {s->ncell, s->ncell, s->ncell, s->ncell, s->ncorn};
  for (int i = 0; i < 5; ++i) {
    if (!views[i]) continue;
    nh_status st = check_view(s, views[i], counts[i]);
    if (st != NH_OK) return st;
    const char* a = static_cast<const char*>(views[i]);
    for (int j = 0; j < i; ++j) {
      if (!views[j]) continue;
      const char* b = static_cast<const char*>(views[j]);
      if (a < b + counts[j] * s->esize && b < a + counts[i] * s->esize)
        return fail(NH_EINVAL, "bound views overlap");
    }
  }
  // no queued work may still use the buffers about to be replaced, and the
  // contents are checked before anything is adopted
  HIP_TRY(hipStreamSynchronize(s->stream));
  HIP_TRY(hipMemsetAsync(s->flags, 0, sizeof(int), s->stream));
  // the bound h is a depth (FP64) or s = h - max(H, 0) (FP32 bulk): checked
  // as a depth against the bathymetry it will be used with
  const void* Hcheck = s->fp32 ? (v->H ? v->H : s->H) : nullptr;
  for (int i = 0; i < 5; ++i) {
    if (!views[i]) continue;
    const int neg = i == 1 ? 16 : 0;  // depth >= 0
    if (s->fp32)
      check_values<float>(s, views[i], counts[i], 8, neg,
                          i == 1 ? Hcheck : nullptr);
    else
      check_values<double>(s, views[i], counts[i], 8, neg);
  }
  int flags = 0;
  HIP_TRY(hipMemcpyAsync(&flags, s->flags, sizeof(int), hipMemcpyDeviceToHost,
                         s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  HIP_TRY(hipMemsetAsync(s->flags, 0, sizeof(int), s->stream));
  if (flags & 8) return fail(NH_EINVAL, "non-finite values in a bound view");
  if (flags & 16) return fail(NH_ENEGDEPTH, "negative depth in the bound h");
  if (v->H) {
    release_own(s, s->H);
    s->H = v->H;
    s->have_H = true;
    if (s->fp32) {  // the bound bathymetry is the FP32 one
      s->H_host.resize(s->ncell);
      nh_status sd = download(s, s->H_host.data(), s->H, s->ncell);
      if (sd != NH_OK) return sd;
    }
  }
  if (!state) return NH_OK;
  release_own(s, s->h);
  s->h = v->h;
  release_own(s, s->q1);
  s->q1 = v->hu;
  if (v->hv) {
    release_own(s, s->q2);
    s->q2 = v->hv;
  } else {
    HIP_TRY(hipMemsetAsync(s->q2, 0, s->ncell * s->esize, s->stream));
  }
  if (v->w) {
    release_own(s, s->w);
    s->w = v->w;
  } else {
    HIP_TRY(hipMemsetAsync(s->w, 0, s->ncorn * s->esize, s->stream));
  }
  return adopt_state(s, nullptr);
}

nh_status nh_step(nh_solver* s, double* dt_used) {
  if (!s) return fail(NH_EINVAL, "null solver");
  if (!s->have_state) return fail(NH_ESTATE, "no valid state (set_state)");
  if (!(s->st.dt_next > 0)) return fail(NH_ESTATE, "dt is not positive");
  nh_status st =
      s->fp32 ? step_impl<float>(s) : step_impl<double>(s);
  nh_status ss = sync_stats(s);
  if (dt_used) *dt_used = s->st.dt_last;
  if (ss != NH_OK) return ss;
  return st;
}

nh_status nh_run(nh_solver* s, int64_t nsteps) {
  if (!s) return fail(NH_EINVAL, "null solver");
  if (nsteps < 0) return fail(NH_EINVAL, "nsteps < 0");
  if (!s->have_state) return fail(NH_ESTATE, "no valid state (set_state)");
  if (!(s->st.dt_next > 0)) return fail(NH_ESTATE, "dt is not positive");
  // steps are queued back to back; the status (non-finite state, no wet
  // cell) is read every kStatusEvery steps and at the end
  const int64_t kStatusEvery = 64;
  for (int64_t n = 0; n < nsteps; ++n) {
    nh_status st = s->fp32 ? step_impl<float>(s) : step_impl<double>(s);
    if (st != NH_OK) {
      nh_status ss = sync_stats(s);
      return ss != NH_OK ? ss : st;
    }
    if ((n + 1) % kStatusEvery == 0 || n + 1 == nsteps) {
      nh_status ss = sync_stats(s);
      if (ss != NH_OK) return ss;
    }
  }
  return NH_OK;
}

nh_status nh_read_state(nh_solver* s, double* h, double* hu, double* hv,
                        double* w, double* p) {
  if (!s) return fail(NH_EINVAL, "null solver");
  nh_status st;
  if (h && (st = download_depth(s, h, s->h, s->ncell)) != NH_OK) return st;
  if (hu && (st = download(s, hu, s->q1, s->ncell)) != NH_OK) return st;
  if (hv) {
    if (s->one_d)
      std::memset(hv, 0, s->ncell * sizeof(double));
    else if ((st = download(s, hv, s->q2, s->ncell)) != NH_OK)
      return st;
  }
  if (w && (st = download(s, w, s->w, s->ncorn)) != NH_OK) return st;
  if (p) {
    HIP_TRY(hipMemcpyAsync(p, s->pcur_ptr(),
                           s->ncorn * sizeof(double), hipMemcpyDeviceToHost,
                           s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
  }
  return NH_OK;
}

nh_status nh_get_stats(const nh_solver* s, nh_stats* out) {
  if (!s || !out) return fail(NH_EINVAL, "null argument");
  *out = s->st;
  out->adjoint_sweeps = s->adj_sweeps_last;
  return NH_OK;
}

nh_status nh_profile(nh_solver* s, int32_t on) {
  if (!s) return fail(NH_EINVAL, "null solver");
  if (s->stream) HIP_TRY(hipStreamSynchronize(s->stream));
  s->prof.flush();
  s->prof.on = on > 0;
  s->prof.sample = on > 1 ? on : 1;
  s->prof.nbatch = 0;
  s->prof.nsolve = 0;
  if (s->prof.on) {
    std::memset(&s->prof.pr, 0, sizeof(s->prof.pr));
    if (s->dstats) {
      HIP_TRY(hipMemsetAsync(&s->dstats->prof_sweeps, 0, sizeof(long long),
                             s->stream));
      HIP_TRY(hipStreamSynchronize(s->stream));
    }
  }
  return NH_OK;
}

nh_status nh_get_profile(nh_solver* s, nh_profile_t* out) {
  if (!s || !out) return fail(NH_EINVAL, "null argument");
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->prof.flush();
  *out = s->prof.pr;
  if (s->persist && s->dstats) {
    long long sw = 0;
    HIP_TRY(hipMemcpy(&sw, &s->dstats->prof_sweeps, sizeof(sw),
                      hipMemcpyDeviceToHost));
    out->solve_kernel_sweeps = sw;
  }
  return NH_OK;
}

void nh_destroy(nh_solver* s) {
  if (!s) return;
  if (s->stream) hipStreamSynchronize(s->stream);
  for (void* p : s->allocs) hipFree(p);
  if (s->slot) hipHostFree(s->slot);
  s->prof.release();
  adj_release(s->adj);
  if (s->own_stream) hipStreamDestroy(s->stream);
  delete s;
}

}  // extern "C"

// ensembles of grids (nh_ensemble_*), built on the pieces above
#include "ensemble_impl.hpp"
// gradients by the adjoint time step (nh_adjoint_run)
#include "adjoint_impl.hpp"

// ---------------------------------------------------------------------------
// Time steps without allocation (nh_run_noalloc): the kernels and host steps
// of nh_run on a solver that lives on the host stack, with the caller's
// device buffers as H and U^n and every other array carved from `scratch`.
// ---------------------------------------------------------------------------
#include <mutex>

namespace {

constexpr size_t kScratchBytes = (size_t)NH_NOALLOC_SCRATCH_BYTES;

// every intermediate array of nh_run_noalloc; each device holds its own copy
// for the life of the process.  In host code this name is only a handle for
// hipGetSymbolAddress: kernels get the address it returns.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_dev[kMaxDevices] = {};

// device address of the current device's scratch, looked up on the first
// call on that device (with it current)
nh_status scratch_address(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices)
    return fail(NH_EDEVICE, "device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return fail(NH_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                  hipGetErrorString(e));
    }
    g_scratch_dev[dev] = static_cast<unsigned char*>(ptr);
  }
  *out = g_scratch_dev[dev];
  return NH_OK;
}

// consecutive 256-byte aligned pieces of the scratch; `used` may run past the
// capacity, which the caller checks before any piece is touched
struct Carver {
  unsigned char* base;
  size_t used = 0;
  void* take(size_t bytes) {
    used = (used + 255) & ~(size_t)255;
    void* p = base + used;
    used += bytes;
    return p;
  }
};

}  // namespace

extern "C" nh_status nh_run_noalloc(const nh_grid* grid,
                                    const nh_params* params, void* hip_stream,
                                    const void* H, void* h, void* hu, void* hv,
                                    void* w, double* p, int64_t nsteps,
                                    nh_stats* stats) {
  nh_status st = check_params(grid, params);
  if (st != NH_OK) return st;
  const bool one_d = grid->ny == 1;
  if (!H || !h || !hu || (!one_d && !hv) || !w || !p)
    return fail(NH_EINVAL, "null device buffer");
  if (nsteps < 0) return fail(NH_EINVAL, "nsteps < 0");
  if (params->solve_path == 2)
    return fail(NH_EINVAL, "nh_run_noalloc solves with launches of 8 sweeps "
                           "(solve_path 0 or 1)");
  if (params->solve_norm != 0)
    return fail(NH_EINVAL, "nh_run_noalloc stops on the measure of eq. (32) "
                           "(solve_norm 0)");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  unsigned char* base = nullptr;
  if ((st = scratch_address(dev, &base)) != NH_OK) return st;

  nh_solver s;  // host stack: no heap, no device allocation
  s.grid = *grid;
  s.par = *params;
  s.par.omega_schedule = nullptr;
  const bool sched = params->omega_schedule && params->n_omega > 0;
  s.nom = sched ? params->n_omega : 1;
  s.one_d = one_d;
  s.fp32 = params->precision == NH_FP32;
  s.esize = s.fp32 ? 4 : 8;
  s.stream = (hipStream_t)hip_stream;
  s.device = dev;
  s.ncell = (long)grid->nx * grid->ny;
  s.ncorn = (long)(grid->nx + 1) * (one_d ? 1 : grid->ny + 1);
  if ((st = choose_sweep_tiles(&s)) != NH_OK) return st;

  const size_t cb = s.ncell * s.esize, kb = s.ncorn * s.esize;
  const size_t kd = s.ncorn * sizeof(double);
  Carver c{base};
  for (void** a : {&s.hs, &s.q1s, &s.q2s, &s.h1, &s.q11, &s.q21})
    *a = c.take(cb);
  if (params->breaking_on)
    for (void** a : {&s.q1b, &s.q2b, &s.rw}) *a = c.take(cb);
  if (one_d) s.q2 = c.take(cb);  // hv is not used in 1D: zeros
  s.w1 = c.take(kb);
  if (params->breaking_on) s.ws = c.take(kb);
  if (params->w_advection) s.wadv = c.take(kb);
  for (void** a : {&s.cdiag, &s.cE, &s.cW, &s.cN, &s.cS, &s.crhs})
    *a = c.take(kb);
  for (void** a : {&s.pa, &s.pb, &s.pc}) *a = c.take(kd);
  if (one_d) {
    s.thomas_cp = (double*)c.take(kd);
    s.thomas_dp = (double*)c.take(kd);
    s.thomas_bb = (double*)c.take(kd);
    s.thomas_z = (double*)c.take(kd);
  }
  s.dt = (double*)c.take(sizeof(double));
  s.lampart = (double*)c.take(nblocks(std::max(s.ncell, s.ncorn)) *
                              sizeof(double));
  s.part = (double*)c.take((size_t)s.ntx * s.nty * sizeof(double));
  s.part_list = (double**)c.take(sizeof(double*));
  s.ntiles_list = (int*)c.take(sizeof(int));
  s.omega_dev = (double*)c.take(s.nom * sizeof(double));
  s.clamped = (double*)c.take(sizeof(double));
  s.flags = (int*)c.take(sizeof(int));
  s.dstats = (nh::DevStats*)c.take(sizeof(nh::DevStats));
  s.slot_dev = (HostSlot*)c.take(sizeof(HostSlot));
  if (c.used > kScratchBytes)
    return fail(NH_EINVAL, "grid needs " + std::to_string(c.used) +
                               " bytes of scratch; the limit is " +
                               std::to_string(kScratchBytes));
  s.slot = nullptr;  // measures are read back by copy (wait_measure)
  s.E_dev = &s.slot_dev->E[0];
  s.H = const_cast<void*>(H);
  s.h = h;
  s.q1 = hu;
  if (!one_d) s.q2 = hv;
  s.w = w;

  // the scratch keeps the previous call's contents: start from zeros
  HIP_TRY(hipMemsetAsync(base, 0, c.used, s.stream));
  const double one = 1.0;
  double* part_h = s.part;
  const int ntiles_h = s.ntx * s.nty;
  HIP_TRY(hipMemcpyAsync(s.omega_dev, sched ? params->omega_schedule : &one,
                         s.nom * sizeof(double), hipMemcpyHostToDevice,
                         s.stream));
  HIP_TRY(hipMemcpyAsync(s.part_list, &part_h, sizeof(double*),
                         hipMemcpyHostToDevice, s.stream));
  HIP_TRY(hipMemcpyAsync(s.ntiles_list, &ntiles_h, sizeof(int),
                         hipMemcpyHostToDevice, s.stream));
  // the state is checked on the device as a bound view is (finite, h >= 0)
  const void* views[5] = {H, h, hu, one_d ? nullptr : hv, w};
  const long counts[5] = {s.ncell, s.ncell, s.ncell, s.ncell, s.ncorn};
  for (int i = 0; i < 5; ++i) {
    if (!views[i]) continue;
    const int neg = i == 1 ? 16 : 0;
    if (s.fp32)
      check_values<float>(&s, views[i], counts[i], 8, neg,
                          i == 1 ? H : nullptr);
    else
      check_values<double>(&s, views[i], counts[i], 8, neg);
  }
  int flags = 0;
  HIP_TRY(hipMemcpyAsync(&flags, s.flags, sizeof(int), hipMemcpyDeviceToHost,
                         s.stream));
  HIP_TRY(hipStreamSynchronize(s.stream));
  if (flags & 8) return fail(NH_EINVAL, "non-finite values in a device buffer");
  if (flags & 16) return fail(NH_ENEGDEPTH, "negative depth in h");
  s.have_H = true;
  if ((st = adopt_state(&s, p, true)) != NH_OK) return st;
  if (!(s.st.dt_next > 0)) return fail(NH_ESTATE, "dt is not positive");

  // nsteps steps, as nh_run queues them
  const int64_t kStatusEvery = 64;
  nh_status result = NH_OK;
  for (int64_t n = 0; n < nsteps; ++n) {
    nh_status sn = s.fp32 ? step_impl<float>(&s) : step_impl<double>(&s);
    if (sn != NH_OK) {
      nh_status ss = sync_stats(&s);
      result = ss != NH_OK ? ss : sn;
      break;
    }
    if ((n + 1) % kStatusEvery == 0 || n + 1 == nsteps) {
      nh_status ss = sync_stats(&s);
      if (ss != NH_OK) {
        result = ss;
        break;
      }
    }
  }
  // the pressure of the last solve (the next call's warm start)
  HIP_TRY(hipMemcpyAsync(p, s.pcur_ptr(), kd, hipMemcpyDeviceToDevice,
                         s.stream));
  HIP_TRY(hipStreamSynchronize(s.stream));
  if (stats) *stats = s.st;
  return result;
}
