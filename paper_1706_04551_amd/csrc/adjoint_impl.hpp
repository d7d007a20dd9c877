// adjoint_impl.hpp -- gradient of a gauge misfit by the adjoint of the time
// stepper (part of the nhswe.hip translation unit; see include/nhswe.h).
//
// Forward: nsteps steps of the solver from its current state with its fixed
// dt, the misfit accumulated on the device after every step, the state
// checkpointed every ckpt_every steps.  Reverse: segment by segment from the
// last, the forward steps of the segment are run again from its checkpoint
// while the stage inputs and both stage pressures are recorded (the tape),
// then the adjoint is carried back through the segment's steps.  Memory:
// checkpoints (nsteps/ckpt_every states) plus one segment of tape.

struct AdjWork {
  std::vector<void*> allocs;
  size_t esize = 8;
  long ncell = 0, ncorn = 0;
  int64_t nsteps = 0;
  int ce = 0, ng = 0, nck = 0;
  // adjoint variables (bulk type)
  void *Lh = nullptr, *Lq1 = nullptr, *Lq2 = nullptr, *Lw = nullptr,
       *LH = nullptr;
  void *L2h = nullptr, *L2q1 = nullptr, *L2q2 = nullptr, *L2w = nullptr;
  void *L1h = nullptr, *L1q1 = nullptr, *L1q2 = nullptr, *Lw1 = nullptr;
  void *Lqs1 = nullptr, *Lqs2 = nullptr, *pbar = nullptr;
  void *tE = nullptr, *tW = nullptr, *tN = nullptr, *tS = nullptr;
  double* mu[2][3] = {};
  void* rowbar = nullptr;  // kRowBars planes of corner cotangents (bulk type)
  void *fpre_h = nullptr, *fpre_q1 = nullptr, *fpre_q2 = nullptr;  // friction
  int mucur[2] = {0, 0};
  // tape of one segment and the checkpoints
  void* tape = nullptr;      // ce x (h, q1, q2, w) bulk + ce x (p1, p2) FP64
  void* ckpt = nullptr;      // (nck + 1) x (h, q1, q2, w) bulk + p FP64
  int* gauges = nullptr;
  double *target = nullptr, *res = nullptr, *J = nullptr;
  double* spart = nullptr;   // per-workgroup scaled maxima
  double** spart_list = nullptr;
  int* spart_n = nullptr;
  double* clamp = nullptr;   // clamped mass of recomputed stages (unused)
};

void adj_release(AdjWork* w) {
  if (!w) return;
  for (void* p : w->allocs) hipFree(p);
  delete w;
}

namespace {

nh_status adj_alloc(AdjWork* w, void** p, size_t bytes, hipStream_t st) {
  if (hipMalloc(p, bytes) != hipSuccess) {
    // the runtime keeps the failure as the thread's last error, which the
    // caller's next check (torch's, after a launch) would report as its own
    (void)hipGetLastError();
    *p = nullptr;
    return fail(NH_ENOMEM, "hipMalloc failed (adjoint buffers)");
  }
  w->allocs.push_back(*p);
  hipMemsetAsync(*p, 0, bytes, st);
  return NH_OK;
}

inline size_t rec_bytes(const nh_solver* s, int np);

nh_status adj_alloc_all(nh_solver* s, AdjWork* w, int64_t nsteps, int ce,
                        int ng);

// (re)allocate the adjoint work space for this run's sizes.  The solver
// keeps a work space only once every buffer of it is allocated: after a
// failed allocation it holds none, so a later call allocates again.
nh_status adj_prepare(nh_solver* s, int64_t nsteps, int ce, int ng) {
  AdjWork* w = s->adj;
  if (w && w->nsteps == nsteps && w->ce == ce && w->ng == ng) return NH_OK;
  adj_release(w);
  s->adj = nullptr;
  w = new AdjWork();
  nh_status r = adj_alloc_all(s, w, nsteps, ce, ng);
  if (r != NH_OK) {
    (void)hipStreamSynchronize(s->stream);
    adj_release(w);
    return r;
  }
  s->adj = w;
  return NH_OK;
}

nh_status adj_alloc_all(nh_solver* s, AdjWork* w, int64_t nsteps, int ce,
                        int ng) {
  const int nck = (int)((nsteps + ce - 1) / ce);
  w->esize = s->esize;
  w->ncell = s->ncell;
  w->ncorn = s->ncorn;
  w->nsteps = nsteps;
  w->ce = ce;
  w->ng = ng;
  w->nck = nck;
  const size_t cb = s->ncell * s->esize, kb = s->ncorn * s->esize,
               kd = s->ncorn * sizeof(double);
  hipStream_t st = s->stream;
  nh_status r = NH_OK;
  void** cells[] = {&w->Lh,   &w->Lq1,  &w->Lq2,    &w->LH,
                    &w->L2h,  &w->L2q1, &w->L2q2,   &w->L1h,
                    &w->L1q1, &w->L1q2, &w->Lqs1,   &w->Lqs2,
                    &w->fpre_h, &w->fpre_q1, &w->fpre_q2};
  void** corners[] = {&w->Lw, &w->L2w, &w->Lw1, &w->pbar,
                      &w->tE, &w->tW,  &w->tN,  &w->tS};
  for (auto c : cells)
    if ((r = adj_alloc(w, c, cb, st)) != NH_OK) return r;
  for (auto c : corners)
    if ((r = adj_alloc(w, c, kb, st)) != NH_OK) return r;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 3; ++b)
      if ((r = adj_alloc(w, (void**)&w->mu[a][b], kd, st)) != NH_OK) return r;
  if ((r = adj_alloc(w, &w->rowbar, nh::kRowBars * kb, st)) != NH_OK)
    return r;
  if ((r = adj_alloc(w, &w->tape, (size_t)ce * rec_bytes(s, 2), st)) !=
          NH_OK ||
      (r = adj_alloc(w, &w->ckpt, (size_t)(nck + 1) * rec_bytes(s, 1), st)) !=
          NH_OK ||
      (r = adj_alloc(w, (void**)&w->gauges, (size_t)ng * sizeof(int), st)) !=
          NH_OK ||
      (r = adj_alloc(w, (void**)&w->target,
                     (size_t)nsteps * ng * sizeof(double), st)) != NH_OK ||
      (r = adj_alloc(w, (void**)&w->res, (size_t)nsteps * ng * sizeof(double),
                     st)) != NH_OK ||
      (r = adj_alloc(w, (void**)&w->J, sizeof(double), st)) != NH_OK ||
      (r = adj_alloc(w, (void**)&w->spart,
                     nblocks(s->ncorn) * sizeof(double), st)) != NH_OK ||
      (r = adj_alloc(w, (void**)&w->spart_list, sizeof(double*), st)) !=
          NH_OK ||
      (r = adj_alloc(w, (void**)&w->spart_n, sizeof(int), st)) != NH_OK ||
      (r = adj_alloc(w, (void**)&w->clamp, sizeof(double), st)) != NH_OK)
    return r;
  int nb = (int)nblocks(s->ncorn);
  HIP_TRY(hipMemcpyAsync(w->spart_list, &w->spart, sizeof(double*),
                         hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(w->spart_n, &nb, sizeof(int), hipMemcpyHostToDevice,
                         st));
  HIP_TRY(hipStreamSynchronize(st));
  return NH_OK;
}

// views of a recorded state (h, q1, q2, w [, p...]) in a packed block
struct StateRec {
  void *h, *q1, *q2, *w;
  double* p;  // checkpoint: warm start; tape: p of stage 1, then stage 2
};

// sizes of the arrays of a record, each rounded up to 256 bytes
inline size_t al256(size_t b) { return (b + 255) & ~size_t(255); }
inline size_t rec_bytes(const nh_solver* s, int np) {
  return 3 * al256(s->ncell * s->esize) + al256(s->ncorn * s->esize) +
         np * al256(s->ncorn * sizeof(double));
}

StateRec rec_at(const nh_solver* s, void* base, size_t index, int np) {
  const size_t cb = al256(s->ncell * s->esize),
               kb = al256(s->ncorn * s->esize);
  char* b = static_cast<char*>(base) + index * rec_bytes(s, np);
  return StateRec{b, b + cb, b + 2 * cb, b + 3 * cb, (double*)(b + 3 * cb + kb)};
}

// the second pressure of a tape record
inline double* rec_p2(const nh_solver* s, const StateRec& r) {
  return (double*)((char*)r.p + al256(s->ncorn * sizeof(double)));
}

nh_status copy_state(nh_solver* s, const StateRec& from_or_to, bool save) {
  const size_t cb = s->ncell * s->esize, kb = s->ncorn * s->esize,
               kd = s->ncorn * sizeof(double);
  auto cp = [&](void* dst, const void* src, size_t n) {
    return hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToDevice, s->stream);
  };
  const StateRec& r = from_or_to;
  if (save) {
    HIP_TRY(cp(r.h, s->h, cb));
    HIP_TRY(cp(r.q1, s->q1, cb));
    HIP_TRY(cp(r.q2, s->q2, cb));
    HIP_TRY(cp(r.w, s->w, kb));
    if (r.p) HIP_TRY(cp(r.p, s->pcur_ptr(), kd));
  } else {
    HIP_TRY(cp(s->h, r.h, cb));
    HIP_TRY(cp(s->q1, r.q1, cb));
    HIP_TRY(cp(s->q2, r.q2, cb));
    HIP_TRY(cp(s->w, r.w, kb));
    if (r.p) {
      s->pcur = 0;
      HIP_TRY(cp(s->pa, r.p, kd));
    }
  }
  return NH_OK;
}

template <typename T>
void fill0(nh_solver* s, void* a, long n) {
  hipLaunchKernelGGL((nh::k_fill<T>), dim3(nblocks(n)), dim3(nh::kBlock), 0,
                     s->stream, n, T(0), (T*)a);
}

// Adjoint of the transposed solve: A^T mu = pbar with the solver's
// relaxation schedule, from the previous mu of this stage; the stop measure
// is relative to max |pbar / diag|.
template <typename T>
nh_status adj_solve(nh_solver* s, AdjWork* w, int stage, double rel_tol,
                    int32_t* sweeps) {
  const long nk = s->ncorn;
  hipLaunchKernelGGL((nh::k_transpose_rows<T>), dim3(nblocks(nk)),
                     dim3(nh::kBlock), 0, s->stream, s->grid.nx, s->grid.ny,
                     (const T*)s->cE, (const T*)s->cW, (const T*)s->cN,
                     (const T*)s->cS, (T*)w->tE, (T*)w->tW, (T*)w->tN,
                     (T*)w->tS);
  hipLaunchKernelGGL((nh::k_scaled_max<T>), dim3(nblocks(nk)),
                     dim3(nh::kBlock), 0, s->stream, (int)nk,
                     (const T*)w->pbar, (const T*)s->cdiag, w->spart);
  ++s->seq;
  hipLaunchKernelGGL(nh::k_reduce_measure, dim3(1), dim3(nh::kBlock), 0,
                     s->stream, (const double* const*)w->spart_list,
                     (const int*)w->spart_n, 1, s->E_dev, &s->slot_dev->seq,
                     s->seq, (const double*)nullptr);
  double scale = 0.0;
  nh_status st = wait_measure(s, &scale);
  if (st != NH_OK) return st;
  *sweeps = 0;
  if (!(scale > 0.0)) {  // no forcing: mu = 0
    fill0<double>(s, w->mu[stage][w->mucur[stage]], nk);
    return NH_OK;
  }
  SysView V{s->cdiag, w->tE, w->tW, w->tN, w->tS, w->pbar,
            {w->mu[stage][0], w->mu[stage][1], w->mu[stage][2]}};
  double measure = 0.0;
  st = solve2d<T>(s, V, w->mucur[stage], rel_tol * scale, sweeps, &measure);
  if (st == NH_ENOCONV) st = NH_OK;  // capped solves are counted, not fatal
  return st;
}

// one forward step with its stage pressures recorded
template <typename T>
nh_status adj_forward_step(nh_solver* s, double* p1, double* p2) {
  s->tape_p[0] = p1;
  s->tape_p[1] = p2;
  nh_status st = step_impl<T>(s);
  s->tape_p[0] = s->tape_p[1] = nullptr;
  if (st == NH_ENOCONV) st = NH_OK;
  return st;
}

// The adjoint of one step: on entry w->L* hold the adjoint of U^{n+1},
// w^{n+1}; on exit that of U^n, w^n.  R is the tape record of step n.
template <typename T>
nh_status adj_step(nh_solver* s, AdjWork* w, const StateRec& R, double tol,
                   int64_t* sweeps_total) {
  const auto& gr = s->grid;
  const auto& pr = s->par;
  hipStream_t st = s->stream;
  const long nc = s->ncell, nk = s->ncorn;
  const dim3 B(nh::kBlock), Gc(nblocks(nc)), Gk(nblocks(nk));
  double* p1 = R.p;
  double* p2 = rec_p2(s, R);
  auto P = [](void* a) { return static_cast<T*>(a); };
  auto C = [](void* a) { return static_cast<const T*>(a); };
  nh::AdjGeom G{gr.nx, gr.ny, gr.dx, gr.dy, pr.g, pr.delta, pr.dry_eps, s->dt};
  const T fric = (T)(pr.g * pr.manning * pr.manning);  // as the forward's
  // --- recompute the stages: FV1 -> (hs, q1s, q2s), correction 1 -> U^(1)
  //     = (hs, q11, q21), w1; FV2 -> (h1, q1b, q2b)
  nh::FvArgs<T> f1{gr.nx, gr.ny, (T)gr.dx, (T)gr.dy, (T)pr.g, (T)pr.delta,
                   (T)pr.dry_eps, P(R.h), P(R.q1), P(R.q2), P(s->H), s->dt,
                   P(s->hs), P(s->q1s), P(s->q2s), w->clamp, fric};
  hipLaunchKernelGGL((nh::k_fv<T, false>), dim3(f1.nblocks()), B, 0, st, f1);
  if (pr.nh_on) {
    nh::CorrectArgs<T> c1{gr.nx, gr.ny, (T)gr.dx, (T)gr.dy, (T)pr.g,
                          (T)pr.delta, (T)pr.dry_eps, 1, P(s->hs), P(s->q1s),
                          P(s->q2s), P(s->H), P(R.w), p1, s->dt, P(s->q11),
                          P(s->q21), P(s->w1), nullptr, nullptr, nullptr,
                          s->lampart, s->flags};
    hipLaunchKernelGGL((nh::k_correct<T, false, false>),
                       dim3(c1.nblocks(false)), B, 0, st, c1);
  } else {
    hipLaunchKernelGGL((nh::k_copy<T>), Gc, B, 0, st, nc, C(s->q1s), P(s->q11));
    hipLaunchKernelGGL((nh::k_copy<T>), Gc, B, 0, st, nc, C(s->q2s), P(s->q21));
    hipLaunchKernelGGL((nh::k_copy<T>), Gk, B, 0, st, nk, C(R.w), P(s->w1));
  }
  nh::FvArgs<T> f2{gr.nx, gr.ny, (T)gr.dx, (T)gr.dy, (T)pr.g, (T)pr.delta,
                   (T)pr.dry_eps, P(s->hs), P(s->q11), P(s->q21), P(s->H),
                   s->dt, P(s->h1), P(s->q1b), P(s->q2b), w->clamp, fric};
  hipLaunchKernelGGL((nh::k_fv<T, false>), dim3(f2.nblocks()), B, 0, st, f2);

  // --- RK average: half of the adjoint to U^n directly, half to U^(2)
  hipLaunchKernelGGL((nh::k_adj_half<T>), Gc, B, 0, st, nc, P(w->Lh), P(w->L2h));
  hipLaunchKernelGGL((nh::k_adj_half<T>), Gc, B, 0, st, nc, P(w->Lq1), P(w->L2q1));
  hipLaunchKernelGGL((nh::k_adj_half<T>), Gc, B, 0, st, nc, P(w->Lq2), P(w->L2q2));
  hipLaunchKernelGGL((nh::k_adj_half<T>), Gk, B, 0, st, nk, P(w->Lw), P(w->L2w));

  // one stage backwards: stage input (Vh, Vq1, Vq2, w_in), FV outputs
  // (hs_, q1s_, q2s_), stage pressure p, adjoint of the stage outputs
  // (lh_out = adjoint of h*, lq_out, lw_out); adds the adjoint of the stage
  // input to (lh_in, lq1_in, lq2_in) and lw_in
  auto stage_back = [&](int idx, void* Vh, void* Vq1, void* Vq2, void* w_in,
                        void* hs_, void* q1s_, void* q2s_, double* p,
                        void* lh_out, void* lq1_out, void* lq2_out,
                        void* lw_out, void* lh_in, void* lq1_in, void* lq2_in,
                        void* lw_in) -> nh_status {
    if (pr.nh_on) {
      // correction
      hipLaunchKernelGGL((nh::k_adj_correct_p<T>), Gk, B, 0, st, G, C(hs_),
                         C(s->H), p, C(lq1_out), C(lq2_out), C(lw_out),
                         P(w->pbar));
      hipLaunchKernelGGL((nh::k_adj_correct_h<T>), Gc, B, 0, st, G, C(hs_),
                         C(s->H), p, C(lq1_out), C(lq2_out), C(lw_out),
                         P(lh_out), P(w->LH), P(w->Lqs1), P(w->Lqs2));
      hipLaunchKernelGGL((nh::k_axpy1<T>), Gk, B, 0, st, nk, C(lw_out),
                         P(lw_in));
      // pressure system of the stage, transposed solve, its adjoint
      nh::AssembleArgs<T> a{gr.nx, gr.ny, (T)gr.dx, (T)gr.dy, P(hs_),
                            P(q1s_), P(q2s_), P(s->H), P(w_in), s->dt,
                            P(s->cdiag), P(s->cE), P(s->cW), P(s->cN),
                            P(s->cS), P(s->crhs)};
      hipLaunchKernelGGL((nh::k_assemble2d<T>), dim3(a.nblocks()), B, 0, st, a);
      int32_t sw = 0;
      nh_status r = adj_solve<T>(s, w, idx, tol, &sw);
      if (r != NH_OK) return r;
      *sweeps_total += sw;
      const double* mu = w->mu[idx][w->mucur[idx]];
      hipLaunchKernelGGL((nh::k_adj_row_bars<T>), Gk, B, 0, st, G, C(hs_),
                         C(q1s_), C(q2s_), C(s->H), C(w_in), p, mu,
                         P(w->rowbar), P(lw_in));
      hipLaunchKernelGGL((nh::k_adj_row_gather<T>), Gc, B, 0, st, G,
                         C(w->rowbar), P(lh_out), P(w->Lqs1), P(w->Lqs2),
                         P(w->LH));
    } else {
      hipLaunchKernelGGL((nh::k_copy<T>), Gc, B, 0, st, nc, C(lq1_out),
                         P(w->Lqs1));
      hipLaunchKernelGGL((nh::k_copy<T>), Gc, B, 0, st, nc, C(lq2_out),
                         P(w->Lqs2));
      hipLaunchKernelGGL((nh::k_axpy1<T>), Gk, B, 0, st, nk, C(lw_out),
                         P(lw_in));
    }
    // friction: the stage's pre-friction result again (friction off), then
    // the adjoint of q_out = q / den back to it
    if (fric > T(0)) {
      nh::FvArgs<T> f0{gr.nx, gr.ny, (T)gr.dx, (T)gr.dy, (T)pr.g,
                       (T)pr.delta, (T)pr.dry_eps, P(Vh), P(Vq1), P(Vq2),
                       P(s->H), s->dt, P(w->fpre_h), P(w->fpre_q1),
                       P(w->fpre_q2), w->clamp, T(0)};
      hipLaunchKernelGGL((nh::k_fv<T, false>), dim3(f0.nblocks()), B, 0, st,
                         f0);
      hipLaunchKernelGGL((nh::k_adj_friction<T>), Gc, B, 0, st, G, fric,
                         C(hs_), C(s->H), C(w->fpre_q1), C(w->fpre_q2),
                         P(w->Lqs1), P(w->Lqs2), P(lh_out));
    }
    // finite volumes
    hipLaunchKernelGGL((nh::k_adj_fv<T, 1>), Gc, B, 0, st, G, C(Vh),
                       C(Vq1), C(Vq2), C(s->H), C(hs_), C(lh_out),
                       C(w->Lqs1), C(w->Lqs2), P(lh_in), P(lq1_in),
                       P(lq2_in), P(w->LH));
    hipLaunchKernelGGL((nh::k_adj_fv<T, 2>), Gc, B, 0, st, G, C(Vh),
                       C(Vq1), C(Vq2), C(s->H), C(hs_), C(lh_out),
                       C(w->Lqs1), C(w->Lqs2), P(lh_in), P(lq1_in),
                       P(lq2_in), P(w->LH));
    return NH_OK;
  };

  // stage 2: input U^(1) = (hs, q11, q21), w1; outputs (h1, q1b, q2b), p2
  fill0<T>(s, w->L1h, nc);
  fill0<T>(s, w->L1q1, nc);
  fill0<T>(s, w->L1q2, nc);
  fill0<T>(s, w->Lw1, nk);
  nh_status r = stage_back(1, s->hs, s->q11, s->q21, s->w1, s->h1, s->q1b,
                           s->q2b, p2, w->L2h, w->L2q1, w->L2q2, w->L2w,
                           w->L1h, w->L1q1, w->L1q2, w->Lw1);
  if (r != NH_OK) return r;
  // stage 1: input U^n = tape, w^n; outputs (hs, q1s, q2s), p1; the adjoint
  // of its h* is that of U^(1)'s depth (L1h)
  return stage_back(0, R.h, R.q1, R.q2, R.w, s->hs, s->q1s, s->q2s, p1,
                    w->L1h, w->L1q1, w->L1q2, w->Lw1, w->Lh, w->Lq1, w->Lq2,
                    w->Lw);
}

template <typename T>
nh_status adjoint_impl(nh_solver* s, int64_t N, double adj_tol, double* J,
                       int64_t* adj_sweeps) {
  AdjWork* w = s->adj;
  const int ce = w->ce, ng = w->ng;
  const long nc = s->ncell, nk = s->ncorn;
  // ---- forward with checkpoints and the misfit
  fill0<double>(s, w->J, 1);
  for (int64_t n = 0; n < N; ++n) {
    if (n % ce == 0) {
      nh_status r = copy_state(s, rec_at(s, w->ckpt, n / ce, 1), true);
      if (r != NH_OK) return r;
    }
    nh_status st = step_impl<T>(s);
    if (st != NH_OK && st != NH_ENOCONV) return st;
    hipLaunchKernelGGL((nh::k_gauge_misfit<T>), dim3(1), dim3(64), 0,
                       s->stream, ng, (const int*)w->gauges, (const T*)s->h,
                       (const T*)s->H, w->target + n * ng, w->res + n * ng,
                       w->J);
    if ((n + 1) % 64 == 0) {
      nh_status ss = sync_stats(s);
      if (ss != NH_OK && ss != NH_ENOCONV) return ss;
    }
  }
  {
    nh_status r = copy_state(s, rec_at(s, w->ckpt, w->nck, 1), true);
    if (r != NH_OK) return r;
    nh_status ss = sync_stats(s);
    if (ss != NH_OK && ss != NH_ENOCONV) return ss;
  }
  nh_stats end_stats = s->st;
  HIP_TRY(hipMemcpyAsync(J, w->J, sizeof(double), hipMemcpyDeviceToHost,
                         s->stream));
  // ---- reverse
  for (void* a : {w->Lh, w->Lq1, w->Lq2, w->LH}) fill0<T>(s, a, nc);
  fill0<T>(s, w->Lw, nk);
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 3; ++b) fill0<double>(s, w->mu[a][b], nk);
  w->mucur[0] = w->mucur[1] = 0;
  hipLaunchKernelGGL((nh::k_gauge_source<T>), dim3(1), dim3(64), 0, s->stream,
                     ng, (const int*)w->gauges, w->res + (N - 1) * ng,
                     (T*)w->Lh);
  for (int seg = w->nck - 1; seg >= 0; --seg) {
    const int64_t n0 = (int64_t)seg * ce;
    const int64_t n1 = std::min<int64_t>(N, n0 + ce);
    nh_status r = copy_state(s, rec_at(s, w->ckpt, seg, 1), false);
    if (r != NH_OK) return r;
    for (int64_t n = n0; n < n1; ++n) {
      StateRec tr = rec_at(s, w->tape, n - n0, 2);
      StateRec cur{tr.h, tr.q1, tr.q2, tr.w, nullptr};
      if ((r = copy_state(s, cur, true)) != NH_OK) return r;
      if ((r = adj_forward_step<T>(s, tr.p, rec_p2(s, tr))) != NH_OK)
        return r;
    }
    for (int64_t n = n1 - 1; n >= n0; --n) {
      StateRec tr = rec_at(s, w->tape, n - n0, 2);
      if ((r = adj_step<T>(s, w, tr, adj_tol, adj_sweeps)) != NH_OK) return r;
      if (n >= 1)
        hipLaunchKernelGGL((nh::k_gauge_source<T>), dim3(1), dim3(64), 0,
                           s->stream, ng, (const int*)w->gauges,
                           w->res + (n - 1) * ng, (T*)w->Lh);
    }
    nh_status ss = sync_stats(s);
    if (ss != NH_OK && ss != NH_ENOCONV) return ss;
  }
  // ---- back to the end of the forward run
  nh_status r = copy_state(s, rec_at(s, w->ckpt, w->nck, 1), false);
  if (r != NH_OK) return r;
  nh::DevStats dend{};
  dend.t = end_stats.t;
  dend.dt_last = end_stats.dt_last;
  dend.step = end_stats.step;
  dend.sweeps_total = end_stats.sweeps_total;
  dend.solves_total = end_stats.solves_total;
  dend.noconv = s->noconv_seen;
  dend.measure = end_stats.measure;
  dend.sweeps[0] = end_stats.sweeps[0];
  dend.sweeps[1] = end_stats.sweeps[1];
  dend.nondom_last = end_stats.nondominant;
  HIP_TRY(hipMemcpyAsync(s->dstats, &dend, sizeof(dend),
                         hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->st = end_stats;
  return NH_OK;
}

}  // namespace

extern "C" {

nh_status nh_adjoint_run(nh_solver* s, int64_t nsteps, int32_t ngauges,
                         const int32_t* gauges, const double* target,
                         int32_t ckpt_every, double adj_tol, double* J,
                         double* dJ_dh0, double* dJ_dhu0, double* dJ_dhv0,
                         double* dJ_dH) {
  if (!s || !gauges || !target || !J)
    return fail(NH_EINVAL, "null argument");
  if (s->one_d) return fail(NH_EINVAL, "the adjoint is for 2D grids");
  if (!s->par.fixed_dt)
    return fail(NH_EINVAL, "the adjoint needs a fixed dt (fixed_dt = 1)");
  if (s->par.breaking_on)
    return fail(NH_EINVAL, "the adjoint does not cover the breaking terms");
  if (s->relax_on)
    return fail(NH_EINVAL, "the adjoint does not cover relaxation zones");
  if (s->par.open_sides != 0 || s->par.periodic != 0)
    return fail(NH_EINVAL, "the adjoint covers walls only");
  if (s->par.w_advection != 0)
    return fail(NH_EINVAL, "the adjoint covers the model's w equation only");
  if (s->par.solve_norm != 0)
    return fail(NH_EINVAL,
                "the adjoint's solves stop on the measure of eq. (32) "
                "(solve_norm = 0)");
  if (nsteps < 1 || ngauges < 1 || ckpt_every < 1)
    return fail(NH_EINVAL, "need nsteps, ngauges, ckpt_every >= 1");
  if (!(adj_tol > 0)) return fail(NH_EINVAL, "need adj_tol > 0");
  for (int g = 0; g < ngauges; ++g)
    if (gauges[g] < 0 || gauges[g] >= s->ncell)
      return fail(NH_EINVAL, "gauge cell out of range");
  if (!s->have_state) return fail(NH_ESTATE, "no valid state (set_state)");
  const int ce = (int)std::min<int64_t>(ckpt_every, nsteps);
  nh_status st = adj_prepare(s, nsteps, ce, ngauges);
  if (st != NH_OK) return st;
  AdjWork* w = s->adj;
  HIP_TRY(hipMemcpyAsync(w->gauges, gauges, ngauges * sizeof(int),
                         hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipMemcpyAsync(w->target, target,
                         (size_t)nsteps * ngauges * sizeof(double),
                         hipMemcpyHostToDevice, s->stream));
  int64_t adj_sweeps = 0;
  st = s->fp32 ? adjoint_impl<float>(s, nsteps, adj_tol, J, &adj_sweeps)
               : adjoint_impl<double>(s, nsteps, adj_tol, J, &adj_sweeps);
  if (st != NH_OK) return st;
  nh_status r;
  if (dJ_dh0 && (r = download(s, dJ_dh0, w->Lh, s->ncell)) != NH_OK) return r;
  if (dJ_dhu0 && (r = download(s, dJ_dhu0, w->Lq1, s->ncell)) != NH_OK)
    return r;
  if (dJ_dhv0 && (r = download(s, dJ_dhv0, w->Lq2, s->ncell)) != NH_OK)
    return r;
  if (dJ_dH && (r = download(s, dJ_dH, w->LH, s->ncell)) != NH_OK) return r;
  s->adj_sweeps_last = adj_sweeps;
  return NH_OK;
}

}  // extern "C"
