// ensemble_impl.hpp -- ensembles of independent 2D grids advanced together
// (part of the nhswe.hip translation unit; see include/nhswe.h).
//
// Every phase of a time step is one launch over all members: the batched
// kernels map their workgroups onto the members through per-kernel prefix
// tables of workgroup counts, and every member runs exactly the arithmetic of
// its single-grid launch.  The pressure solves of all members run in
// lockstep relaxation cycles; the checks decide on the device which
// members leave at each convergence check, so the members' results and sweep
// counts are those of their own single-grid solves.  A solve is launches of
// 8 sweeps with the number of members still active read by the host at each
// check, or (solve_path 2) one cooperative launch (k_ens_solve: sweeps and
// checks as phases between grid barriers, no host decision inside).  Each
// member is an nh_solver (its buffers, dt, statistics) bound to the
// ensemble's stream.

// ensemble slot in mapped host memory: sequence number of the last check,
// members still active, per-member measures and active flags
struct EnsSlot {
  long long seq;
  int nactive;
  int pad;
  // followed by double E[n], int active[n]
};

struct nh_ensemble {
  int n = 0;
  bool fp32 = false;
  int sweep_m = nh::kSweepM;   // region points per thread of the batched sweep
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int nh_on = 1, breaking_on = 0, kmax = 0, check_every = 1;
  int solve_path = 0;          // 2: one launch per solve; 0, 1: cycles
  int wait_polls = 0;          // of the one-launch solve's waits
  int persist_grid = 0;        // workgroups of the one-launch solve (0: none)
  // one-launch solve: [0] barrier arrivals, [1] low word: flags, [2..9]
  // item counters
  unsigned long long* psync = nullptr;
  // graph of one step (nh_ensemble_run_graph), captured for the current
  // tables; the solves inside are plain launches (capturing)
  hipGraphExec_t step_graph = nullptr;
  bool capturing = false;
  std::vector<nh_solver*> mem;
  std::vector<int> live;       // members in the batch tables (state set, ok)
  std::vector<char> failed;    // member stopped by an error
  std::vector<nh_status> member_status;
  bool dirty = true;           // tables must be rebuilt

  // device tables, indexed by position in `live`
  void* table = nullptr;       // one allocation holding everything below
  size_t table_bytes = 0;
  void *fv[2] = {}, *brc[2] = {}, *brk[2] = {}, *asmb[2] = {}, *corr[2] = {};
  void *sweep = nullptr, *fin = nullptr;
  int *pre_fv = nullptr, *pre_brc = nullptr, *pre_brk = nullptr,
      *pre_asm = nullptr, *pre_sweep = nullptr, *pre_corr = nullptr;
  int tot_fv = 0, tot_brc = 0, tot_brk = 0, tot_asm = 0, tot_sweep = 0,
      tot_corr = 0;
  size_t sweep_lds = 0;
  std::vector<long> live_corners;  // corners of each live member
  std::vector<int> sweep_nb;       // sweep workgroups of each live member
  int *ids_all = nullptr;          // 0..L-1 (device)
  int *nb_dev = nullptr;           // sweep_nb (device)
  int *act_ids = nullptr, *act_pre = nullptr;  // compacted after a check

  nh::EnsMember* dmem = nullptr;   // per member (all n, not only live)
  nh::EnsMember* dmem_live = nullptr;  // gathered copy for the batch order
  bool live_current = false;       // dmem_live holds the current records
  EnsSlot* slot = nullptr;         // mapped host memory
  EnsSlot* slot_dev = nullptr;
  double* E_host = nullptr;
  int* active_host = nullptr;
  long long seq = 0;
  ProfPool prof;
};

namespace {

double* slot_E(EnsSlot* s) { return reinterpret_cast<double*>(s + 1); }
int* slot_active(EnsSlot* s, int n) {
  return reinterpret_cast<int*>(slot_E(s) + n);
}

// candidate sweep tiles (corners); a tile fits when its region
// (BX+2S)(BY+2S) fits the workgroup's kSweepB * sweep_m points.  FP32-bulk
// ensembles sweep with 3 region points per thread, so that large members
// can take the larger tiles (FP64 keeps 2: its 3-point kernel loses half
// its occupancy)
constexpr int kTiles[][2] = {{24, 24}, {28, 28}, {32, 24}, {40, 16},
                             {48, 16}, {64, 8},  {16, 16}, {32, 32},
                             {36, 28}, {40, 24}};

bool tile_ok(int bx, int by, int points) {
  return bx >= 4 && by >= 4 &&
         (bx + 2 * nh::kSweepS) * (by + 2 * nh::kSweepS) <=
             nh::kSweepB * points;
}

// (re)allocate the per-tile measures for the member's tile shape
nh_status set_member_tile(nh_solver* m, int bx, int by) {
  if (!tile_ok(bx, by, m->sweep_m))
    return fail(NH_EINVAL, "tile does not fit the workgroup");
  int ntx = (m->grid.nx + 1 + bx - 1) / bx;
  int nty = (m->grid.ny + 1 + by - 1) / by;
  if ((long)ntx * nty > (long)m->ntx * m->nty) {
    nh_status st = dalloc(m, (void**)&m->part, (size_t)ntx * nty * sizeof(double));
    if (st != NH_OK) return st;
  }
  m->tbx = bx;
  m->tby = by;
  m->ntx = ntx;
  m->nty = nty;
  return NH_OK;
}

template <typename T>
const void* ens_persist_kernel(int m) {
  if (m == nh::kSweepMBig)
    return (const void*)nh::k_ens_solve<T, nh::kSweepB, nh::kSweepS,
                                        nh::kSweepMBig>;
  return (const void*)nh::k_ens_solve<T, nh::kSweepB, nh::kSweepS,
                                      nh::kSweepM>;
}

// Workgroups of the one-launch solve (solve_path 2): as many as can be
// co-resident (a multiple of 8, so that an item keeps its XCD), at most one
// per item; 0 when the solve runs as launches of 8 sweeps.  The launches of
// 8 sweeps stay the default: on the 64-member workload they are ~11 %
// faster, the one launch reading the iterate at device scope (past the L2)
// where the launches find the tiles' shared halos in L2.
template <typename T>
nh_status ens_persist_grid(nh_ensemble* e) {
  e->persist_grid = 0;
  if (e->solve_path != 2 || e->tot_sweep <= 0) return NH_OK;
  if ((int)e->live.size() > nh::kEnsPersistMax)
    return fail(NH_EINVAL, "solve_path 2: more than 1024 members");
  int dev = 0, coop = 0, cus = 0, per_cu = 0;
  const void* kern = ens_persist_kernel<T>(e->sweep_m);
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch,
                            dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                            dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, kern, nh::kSweepB, e->sweep_lds) != hipSuccess) {
    (void)hipGetLastError();
    coop = 0;
  }
  const long cap = coop ? ((long)per_cu * cus) / 8 * 8 : 0;
  if (cap < 8)
    return fail(NH_EINVAL,
                "solve_path 2: no cooperative launch of the ensemble solve "
                "on this device");
  e->persist_grid = (int)std::min<long>(cap, e->tot_sweep);
  return NH_OK;
}

// Build the batch tables of the live members and upload them (synchronous).
template <typename T>
nh_status ens_build(nh_ensemble* e) {
  const int L = (int)e->live.size();
  if (e->step_graph) {  // captured with the tables about to be replaced
    HIP_TRY(hipGraphExecDestroy(e->step_graph));
    e->step_graph = nullptr;
  }
  std::vector<nh::FvArgs<T>> fv[2];
  std::vector<nh::BreakCellsArgs<T>> brc[2];
  std::vector<nh::BreakCornersArgs<T>> brk[2];
  std::vector<nh::AssembleArgs<T>> asmb[2];
  std::vector<nh::CorrectArgs<T>> corr[2];
  std::vector<nh::SweepArgs<T>> sw;
  std::vector<nh::FinalizeArgs> fin;
  std::vector<int> pre[6];
  int tot[6] = {0, 0, 0, 0, 0, 0};
  e->sweep_lds = 0;
  e->live_corners.clear();
  e->sweep_nb.clear();
  for (int i = 0; i < L; ++i) {
    nh_solver* m = e->mem[e->live[i]];
    for (int st = 0; st < 2; ++st) {
      StagePlan S = stage_plan(m, st);
      fv[st].push_back(Args<T>::fv(m, S));
      brc[st].push_back(Args<T>::break_cells(m, S));
      brk[st].push_back(Args<T>::break_corners(m, S));
      asmb[st].push_back(Args<T>::assemble(m, S));
      corr[st].push_back(Args<T>::correct(m, S, m->pa));
    }
    sw.push_back(Args<T>::sweep(m));
    fin.push_back(finalize_args(m, true));
    const int nb[6] = {fv[0].back().nblocks(), brc[0].back().nblocks(),
                       brk[0].back().nblocks(false), asmb[0].back().nblocks(),
                       sw.back().nblocks(), corr[0].back().nblocks(false)};
    for (int k = 0; k < 6; ++k) {
      pre[k].push_back(tot[k]);
      if ((long)tot[k] + nb[k] > (1L << 30))
        return fail(NH_EINVAL, "ensemble too large for one launch");
      tot[k] += nb[k];
    }
    e->sweep_lds = std::max(e->sweep_lds, sweep_lds_bytes(m->tbx, m->tby));
    e->live_corners.push_back(m->ncorn);
    e->sweep_nb.push_back(nb[4]);
  }
  for (int k = 0; k < 6; ++k) pre[k].push_back(tot[k]);
  // layout: every block 256-byte aligned
  std::vector<char> buf;
  auto put = [&](const void* src, size_t bytes) {
    size_t off = (buf.size() + 255) & ~size_t(255);
    buf.resize(off + bytes);
    if (bytes) std::memcpy(buf.data() + off, src, bytes);
    return off;
  };
  size_t o_fv[2], o_brc[2], o_brk[2], o_asm[2], o_corr[2], o_pre[6];
  for (int st = 0; st < 2; ++st) {
    o_fv[st] = put(fv[st].data(), fv[st].size() * sizeof(fv[st][0]));
    o_brc[st] = put(brc[st].data(), brc[st].size() * sizeof(brc[st][0]));
    o_brk[st] = put(brk[st].data(), brk[st].size() * sizeof(brk[st][0]));
    o_asm[st] = put(asmb[st].data(), asmb[st].size() * sizeof(asmb[st][0]));
    o_corr[st] = put(corr[st].data(), corr[st].size() * sizeof(corr[st][0]));
  }
  size_t o_sw = put(sw.data(), sw.size() * sizeof(sw[0]));
  size_t o_fin = put(fin.data(), fin.size() * sizeof(fin[0]));
  for (int k = 0; k < 6; ++k)
    o_pre[k] = put(pre[k].data(), pre[k].size() * sizeof(int));
  std::vector<int> ids(L);
  for (int i = 0; i < L; ++i) ids[i] = i;
  size_t o_ids = put(ids.data(), L * sizeof(int));
  size_t o_nb = put(e->sweep_nb.data(), L * sizeof(int));
  size_t o_aids = put(ids.data(), L * sizeof(int));
  size_t o_apre = put(pre[4].data(), (L + 1) * sizeof(int));
  if (buf.size() > e->table_bytes) {
    if (e->table) hipFree(e->table);
    e->table = nullptr;
    e->table_bytes = 0;
    if (hipMalloc(&e->table, buf.size()) != hipSuccess)
      return fail(NH_ENOMEM, "allocation of the ensemble tables failed");
    e->table_bytes = buf.size();
  }
  HIP_TRY(hipStreamSynchronize(e->stream));
  HIP_TRY(hipMemcpy(e->table, buf.data(), buf.size(), hipMemcpyHostToDevice));
  char* base = static_cast<char*>(e->table);
  for (int st = 0; st < 2; ++st) {
    e->fv[st] = base + o_fv[st];
    e->brc[st] = base + o_brc[st];
    e->brk[st] = base + o_brk[st];
    e->asmb[st] = base + o_asm[st];
    e->corr[st] = base + o_corr[st];
  }
  e->sweep = base + o_sw;
  e->fin = base + o_fin;
  int** pres[6] = {&e->pre_fv, &e->pre_brc, &e->pre_brk,
                   &e->pre_asm, &e->pre_sweep, &e->pre_corr};
  for (int k = 0; k < 6; ++k) *pres[k] = (int*)(base + o_pre[k]);
  e->ids_all = (int*)(base + o_ids);
  e->nb_dev = (int*)(base + o_nb);
  e->act_ids = (int*)(base + o_aids);
  e->act_pre = (int*)(base + o_apre);
  e->tot_fv = tot[0];
  e->tot_brc = tot[1];
  e->tot_brk = tot[2];
  e->tot_asm = tot[3];
  e->tot_sweep = tot[4];
  e->tot_corr = tot[5];
  nh_status ps = ens_persist_grid<T>(e);
  if (ps != NH_OK) return ps;
  e->dirty = false;
  return NH_OK;
}

// Member records in batch order <-> per-member records.  The batch kernels
// index records by position in `live`; the records of all n members live in
// dmem and are gathered before a run and scattered back after it.
nh_status ens_gather(nh_ensemble* e, bool to_live) {
  if (!to_live && !e->live_current) return NH_OK;
  e->live_current = to_live;
  for (size_t i = 0; i < e->live.size(); ++i) {
    nh::EnsMember* a = e->dmem + e->live[i];
    nh::EnsMember* b = e->dmem_live + i;
    HIP_TRY(hipMemcpyAsync(to_live ? b : a, to_live ? a : b,
                           sizeof(nh::EnsMember), hipMemcpyDeviceToDevice,
                           e->stream));
  }
  return NH_OK;
}

// one batched sweep launch over the members ids[0..n) with workgroup prefix
// pre and `total` workgroups
template <typename T>
void ens_sweeps(nh_ensemble* e, const int* ids, const int* pre, int n,
                int total, bool check, int k0, int nsw, int iin, int iout,
                int isave) {
  if (total <= 0) return;
  nh::SweepLaunch Lc{iin, iout, isave, k0, nsw, check ? 1 : 0,
                     0, nullptr, nullptr, 0};
  const auto* as = (const nh::SweepArgs<T>*)e->sweep;
  const auto* mem = (const nh::EnsMember*)e->dmem_live;
  if (e->sweep_m == nh::kSweepMBig)
    hipLaunchKernelGGL((nh::k_sweep_tb_batch<T, nh::kSweepB, nh::kSweepS,
                                               nh::kSweepMBig>),
                       dim3(total), dim3(nh::kSweepB), e->sweep_lds,
                       e->stream, as, ids, pre, n, mem, Lc);
  else
    hipLaunchKernelGGL((nh::k_sweep_tb_batch<T, nh::kSweepB, nh::kSweepS,
                                               nh::kSweepM>),
                       dim3(total), dim3(nh::kSweepB), e->sweep_lds,
                       e->stream, as, ids, pre, n, mem, Lc);
}

// Lockstep solve of every live member (the same cycle structure as the
// single-grid solve, see solve2d).
template <typename T>
nh_status ens_solve(nh_ensemble* e, int stage) {
  const int L = (int)e->live.size();
  const int ce = e->check_every > 0 ? e->check_every : 1;
  const int kmax = e->kmax;
  const int S = nh::kSweepS;
  const int kAhead = 1;
  hipLaunchKernelGGL(nh::k_ens_begin, dim3(1), dim3(256), 0, e->stream,
                     e->dmem_live, L, e->persist_grid > 0 ? e->psync : nullptr);
  if (e->persist_grid > 0) {
    const auto* as = (const nh::SweepArgs<T>*)e->sweep;
    const int* pre = e->pre_sweep;
    nh::EnsMember* mem = e->dmem_live;
    int Lm = L;
    nh::EnsPersist P{kmax, ce, stage, e->psync, e->psync + 2,
                     reinterpret_cast<int*>(e->psync + 1),
                     wait_bound(e->wait_polls)};
    void* args[] = {(void*)&as, (void*)&pre, (void*)&Lm, (void*)&mem,
                    (void*)&P};
    long pm = e->prof.open(e->stream, 5);
    // a graph takes the solve as a plain launch of the same workgroups (no
    // more than are co-resident; the waits are bounded)
    if (e->capturing)
      HIP_TRY(hipLaunchKernel(ens_persist_kernel<T>(e->sweep_m),
                              dim3(e->persist_grid), dim3(nh::kSweepB), args,
                              e->sweep_lds, e->stream));
    else
      HIP_TRY(hipLaunchCooperativeKernel(ens_persist_kernel<T>(e->sweep_m),
                                         dim3(e->persist_grid),
                                         dim3(nh::kSweepB), args,
                                         e->sweep_lds, e->stream));
    e->prof.close(e->stream, pm, 1);
    return NH_OK;
  }
  int k = 0, cur = 0;
  int* act = e->active_host;
  // launch table: every member for the first check, then the members still
  // active (compacted on the device after each check)
  const int* ids = e->ids_all;
  const int* pre = e->pre_sweep;
  int nmem = L, total = e->tot_sweep;
  for (;;) {
    const int save = (cur + 2) % 3, out = (cur + 1) % 3;
    const int kc = k;
    int nsw = k >= kmax ? 0 : std::min(std::min(S, ce), kmax - k);
    ens_sweeps<T>(e, ids, pre, nmem, total, true, k, nsw, cur, out, save);
    ++e->seq;
    hipLaunchKernelGGL((nh::k_ens_check<T>), dim3(L), dim3(nh::kBlock), 0,
                       e->stream, (const nh::SweepArgs<T>*)e->sweep,
                       e->dmem_live, kc, kmax, save, stage,
                       slot_E(e->slot_dev), slot_active(e->slot_dev, e->n));
    hipLaunchKernelGGL(nh::k_ens_publish, dim3(1), dim3(nh::kBlock), 0,
                       e->stream, (const nh::EnsMember*)e->dmem_live, L,
                       &e->slot_dev->nactive, &e->slot_dev->seq, e->seq);
    if (nsw > 0) {
      cur = out;
      k += nsw;
    }
    int other = 3 - cur - save;
    int queued = 0;
    auto queue_until = [&](int limit) {
      while (k % ce != 0 && k < kmax && queued < limit) {
        int n2 = std::min(std::min(S, ce - k % ce), kmax - k);
        ens_sweeps<T>(e, ids, pre, nmem, total, false, k, n2, cur, other,
                      other);
        std::swap(cur, other);
        k += n2;
        ++queued;
      }
    };
    if (nsw > 0) queue_until(kAhead);
    nh_status ws = wait_seq(e->stream, &e->slot->seq, e->seq);
    if (ws != NH_OK) return ws;
    if (e->slot->nactive == 0) break;
    // the rest of the cycle, over the members still active
    double corners = 0.0;
    nmem = 0;
    total = 0;
    for (int i = 0; i < L; ++i)
      if (act[i]) {
        corners += (double)e->live_corners[i];
        total += e->sweep_nb[i];
        ++nmem;
      }
    hipLaunchKernelGGL(nh::k_ens_compact, dim3(1), dim3(64), 0, e->stream,
                       (const nh::EnsMember*)e->dmem_live,
                       (const int*)e->nb_dev, L, e->act_ids, e->act_pre);
    ids = e->act_ids;
    pre = e->act_pre;
    int before = queued;
    long pm = (k % ce != 0 && k < kmax) ? e->prof.open(e->stream, 4) : -1;
    queue_until(1 << 30);
    e->prof.close(e->stream, pm, queued - before,
                  (double)(queued - before) * S * corners);
  }
  return NH_OK;
}

template <typename T>
nh_status ens_stage(nh_ensemble* e, int idx) {
  const int L = (int)e->live.size();
  hipStream_t st = e->stream;
  const dim3 B(nh::kBlock);
  long pm = e->prof.open(st, 0);
  hipLaunchKernelGGL((nh::k_fv_batch<T, false>), dim3(e->tot_fv), B, 0, st,
                     (const nh::FvArgs<T>*)e->fv[idx], (const int*)e->pre_fv,
                     L);
  e->prof.close(st, pm, 1);
  pm = e->prof.open(st, 1);
  if (e->breaking_on) {
    hipLaunchKernelGGL((nh::k_break_cells_batch<T, false>), dim3(e->tot_brc),
                       B, 0, st, (const nh::BreakCellsArgs<T>*)e->brc[idx],
                       (const int*)e->pre_brc, L);
    hipLaunchKernelGGL((nh::k_break_corners_batch<T, false>),
                       dim3(e->tot_brk), B, 0, st,
                       (const nh::BreakCornersArgs<T>*)e->brk[idx],
                       (const int*)e->pre_brk, L);
  }
  if (e->nh_on)
    hipLaunchKernelGGL((nh::k_assemble2d_batch<T>), dim3(e->tot_asm), B, 0,
                       st, (const nh::AssembleArgs<T>*)e->asmb[idx],
                       (const int*)e->pre_asm, L);
  e->prof.close(st, pm, (e->breaking_on ? 2 : 0) + (e->nh_on ? 1 : 0));
  if (e->nh_on) {
    pm = e->prof.open(st, 2);
    nh_status s2 = ens_solve<T>(e, idx);
    if (s2 != NH_OK) return s2;
    e->prof.close(st, pm, 0);
  }
  pm = e->prof.open(st, 3);
  if (idx == 1)
    hipLaunchKernelGGL((nh::k_correct_batch<T, false, true>),
                       dim3(e->tot_corr), B, 0, st,
                       (const nh::CorrectArgs<T>*)e->corr[idx],
                       (const int*)e->pre_corr, L,
                       (const nh::SweepArgs<T>*)e->sweep,
                       (const nh::EnsMember*)e->dmem_live);
  else
    hipLaunchKernelGGL((nh::k_correct_batch<T, false, false>),
                       dim3(e->tot_corr), B, 0, st,
                       (const nh::CorrectArgs<T>*)e->corr[idx],
                       (const int*)e->pre_corr, L,
                       (const nh::SweepArgs<T>*)e->sweep,
                       (const nh::EnsMember*)e->dmem_live);
  e->prof.close(st, pm, 1);
  return NH_OK;
}

template <typename T>
nh_status ens_step(nh_ensemble* e) {
  nh_status st = ens_stage<T>(e, 0);
  if (st != NH_OK) return st;
  st = ens_stage<T>(e, 1);
  if (st != NH_OK) return st;
  long pm = e->prof.open(e->stream, 3);
  hipLaunchKernelGGL(nh::k_finalize_dt_batch, dim3(e->live.size()),
                     dim3(nh::kBlock), 0, e->stream,
                     (const nh::FinalizeArgs*)e->fin);
  e->prof.close(e->stream, pm, 1);
  return NH_OK;
}

// Statistics of every live member; a member whose state failed leaves the
// batch (its status is kept in member_status).
nh_status ens_sync(nh_ensemble* e) {
  HIP_TRY(hipStreamSynchronize(e->stream));
  int eflags = 0;
  HIP_TRY(hipMemcpy(&eflags, e->psync + 1, sizeof(int), hipMemcpyDeviceToHost));
  if (eflags & nh::kFlagWaitBound)
    return fail(NH_EDEVICE,
                "ensemble solve: a grid barrier wait gave up (workgroups not "
                "co-resident)");
  std::vector<nh::EnsMember> rec(e->live.size());
  if (!rec.empty())
    HIP_TRY(hipMemcpy(rec.data(), e->dmem_live,
                      rec.size() * sizeof(nh::EnsMember),
                      hipMemcpyDeviceToHost));
  e->prof.flush();
  nh_status worst = NH_OK;
  std::vector<int> keep;
  for (size_t i = 0; i < e->live.size(); ++i) {
    const int id = e->live[i];
    nh_solver* m = e->mem[id];
    nh_status st = sync_stats(m);
    m->st.sweeps[0] = rec[i].sweeps[0];
    m->st.sweeps[1] = rec[i].sweeps[1];
    m->st.measure = rec[i].measure;
    m->st.sweeps_total = rec[i].sweeps_total;
    m->st.solves_total = rec[i].solves_total;
    if (st == NH_OK && rec[i].noconv > 0) {
      m->st.last_status = NH_ENOCONV;
    } else if (st == NH_OK) {
      m->st.last_status = NH_OK;
    }
    if (st != NH_OK) {
      e->failed[id] = 1;
      e->member_status[id] = st;
      if (worst == NH_OK) worst = st;
    } else {
      keep.push_back(id);
    }
  }
  if (keep.size() != e->live.size()) {
    // scatter the records, then rebuild the tables without the failed members
    nh_status s2 = ens_gather(e, false);
    if (s2 != NH_OK) return s2;
    e->live = keep;
    e->dirty = true;
  }
  return worst;
}

nh_status ens_check_member(const nh_ensemble* e, int k) {
  if (!e) return fail(NH_EINVAL, "null ensemble");
  if (k < 0 || k >= e->n) return fail(NH_EINVAL, "member index out of range");
  return NH_OK;
}

}  // namespace

extern "C" {

nh_status nh_ensemble_create(int32_t n, const nh_grid* grids,
                             const nh_params* params, void* hip_stream,
                             nh_ensemble** out) {
  if (!out) return fail(NH_EINVAL, "null output pointer");
  *out = nullptr;
  if (n < 1 || !grids || !params) return fail(NH_EINVAL, "need n >= 1 members");
  for (int k = 0; k < n; ++k) {
    nh_status st = check_params(&grids[k], &params[k]);
    if (st != NH_OK) return st;
    if (grids[k].ny < 2) return fail(NH_EINVAL, "ensemble members must be 2D");
    if (params[k].w_advection != 0)
      return fail(NH_EINVAL,
                  "ensemble members use the model's w equation "
                  "(w_advection = 0)");
    if (params[k].solve_norm != 0)
      return fail(NH_EINVAL,
                  "ensemble members stop on the measure of eq. (32) "
                  "(solve_norm = 0)");
    const nh_params& a = params[0];
    const nh_params& b = params[k];
    if (a.precision != b.precision || a.nh_on != b.nh_on ||
        a.breaking_on != b.breaking_on ||
        a.solve_max_iter != b.solve_max_iter ||
        a.solve_path != b.solve_path ||
        (a.check_every > 0 ? a.check_every : 1) !=
            (b.check_every > 0 ? b.check_every : 1))
      return fail(NH_EINVAL,
                  "members must share precision, nh_on, breaking_on, "
                  "solve_max_iter, solve_path and check_every");
  }
  nh_ensemble* e = new nh_ensemble();
  e->n = n;
  e->fp32 = params[0].precision == NH_FP32;
  e->sweep_m = e->fp32 ? nh::kSweepMBig : nh::kSweepM;
  e->nh_on = params[0].nh_on;
  e->breaking_on = params[0].breaking_on;
  e->kmax = params[0].solve_max_iter;
  e->check_every = params[0].check_every > 0 ? params[0].check_every : 1;
  e->solve_path = params[0].solve_path;
  e->wait_polls = params[0].wait_polls;
  if (hip_stream) {
    e->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreate(&e->stream) != hipSuccess) {
      delete e;
      return fail(NH_EDEVICE, "hipStreamCreate failed");
    }
    e->own_stream = true;
  }
  e->failed.assign(n, 0);
  e->member_status.assign(n, NH_OK);
  for (int k = 0; k < n; ++k) {
    nh_solver* m = nullptr;
    // the member's own solve path is never taken: the ensemble solves it
    nh_params pk = params[k];
    pk.solve_path = 1;
    nh_status st = nh_create(&grids[k], &pk, e->stream, &m);
    if (st != NH_OK) {
      std::string msg = g_err;
      nh_ensemble_destroy(e);
      return fail(st, "member " + std::to_string(k) + ": " + msg);
    }
    m->sweep_m = e->sweep_m;  // members are swept by the batched kernel
    e->mem.push_back(m);
  }
  size_t slot_bytes =
      sizeof(EnsSlot) + (size_t)n * (sizeof(double) + sizeof(int));
  if (hipMalloc((void**)&e->dmem, n * sizeof(nh::EnsMember)) != hipSuccess ||
      hipMalloc((void**)&e->dmem_live, n * sizeof(nh::EnsMember)) !=
          hipSuccess ||
      hipHostMalloc((void**)&e->slot, slot_bytes,
                    hipHostMallocMapped | hipHostMallocCoherent) !=
          hipSuccess ||
      hipHostGetDevicePointer((void**)&e->slot_dev, e->slot, 0) !=
          hipSuccess ||
      hipMalloc((void**)&e->psync, 256) != hipSuccess ||
      hipMemset(e->psync, 0, 256) != hipSuccess) {
    nh_ensemble_destroy(e);
    return fail(NH_ENOMEM, "allocation of the ensemble records failed");
  }
  std::memset(e->slot, 0, slot_bytes);
  e->E_host = slot_E(e->slot);
  e->active_host = slot_active(e->slot, n);
  std::vector<nh::EnsMember> rec(n);
  for (int k = 0; k < n; ++k) {
    std::memset(&rec[k], 0, sizeof(rec[k]));
    rec[k].tol = params[k].solve_tol;
  }
  if (hipMemcpy(e->dmem, rec.data(), n * sizeof(nh::EnsMember),
                hipMemcpyHostToDevice) != hipSuccess) {
    nh_ensemble_destroy(e);
    return fail(NH_EDEVICE, "upload of the ensemble records failed");
  }
  *out = e;
  return NH_OK;
}

nh_status nh_ensemble_set_bathymetry(nh_ensemble* e, int32_t k,
                                     const double* H) {
  nh_status st = ens_check_member(e, k);
  if (st != NH_OK) return st;
  return nh_set_bathymetry(e->mem[k], H);
}

nh_status nh_ensemble_set_state(nh_ensemble* e, int32_t k, const double* h,
                                const double* hu, const double* hv,
                                const double* w, const double* p) {
  nh_status st = ens_check_member(e, k);
  if (st != NH_OK) return st;
  // records of the live members back to their own slots first
  if ((st = ens_gather(e, false)) != NH_OK) return st;
  HIP_TRY(hipStreamSynchronize(e->stream));
  st = nh_set_state(e->mem[k], h, hu, hv, w, p);
  nh::EnsMember rec;
  std::memset(&rec, 0, sizeof(rec));
  rec.tol = e->mem[k]->par.solve_tol;
  HIP_TRY(hipMemcpy(e->dmem + k, &rec, sizeof(rec), hipMemcpyHostToDevice));
  e->failed[k] = st == NH_OK ? 0 : 1;
  e->member_status[k] = st;
  e->live.clear();
  for (int i = 0; i < e->n; ++i)
    if (!e->failed[i] && e->mem[i]->have_state) e->live.push_back(i);
  e->dirty = true;
  return st;
}

nh_status nh_ensemble_set_tile(nh_ensemble* e, int32_t k, int32_t bx,
                               int32_t by) {
  nh_status st = ens_check_member(e, k);
  if (st != NH_OK) return st;
  HIP_TRY(hipStreamSynchronize(e->stream));
  st = set_member_tile(e->mem[k], bx, by);
  e->dirty = true;
  return st;
}

nh_status nh_ensemble_get_tile(const nh_ensemble* e, int32_t k, int32_t* bx,
                               int32_t* by) {
  nh_status st = ens_check_member(e, k);
  if (st != NH_OK) return st;
  if (bx) *bx = e->mem[k]->tbx;
  if (by) *by = e->mem[k]->tby;
  return NH_OK;
}

nh_status nh_ensemble_tune(nh_ensemble* e, int32_t reps) {
  if (!e) return fail(NH_EINVAL, "null ensemble");
  if (reps < 1) reps = 1;
  HIP_TRY(hipStreamSynchronize(e->stream));
  // one timing per distinct grid shape, on scratch data of that shape
  std::vector<std::pair<std::pair<int, int>, std::pair<int, int>>> done;
  hipEvent_t a = nullptr, b = nullptr;
  HIP_TRY(hipEventCreate(&a));
  if (hipEventCreate(&b) != hipSuccess) {
    hipEventDestroy(a);
    return fail(NH_EDEVICE, "hipEventCreate failed");
  }
  nh_status result = NH_OK;
  for (int k = 0; k < e->n && result == NH_OK; ++k) {
    nh_solver* m = e->mem[k];
    std::pair<int, int> shape{m->grid.nx, m->grid.ny};
    int bx = 0, by = 0;
    for (auto& d : done)
      if (d.first == shape) {
        bx = d.second.first;
        by = d.second.second;
      }
    if (bx == 0) {
      // scratch system: diag 1, neighbours 0.25, rhs 0; iterates 0
      const size_t es = m->esize, nk = (size_t)m->ncorn;
      void* scratch = nullptr;
      size_t bytes = 6 * nk * es + 2 * nk * sizeof(double) +
                     8192 * sizeof(double);
      if (hipMalloc(&scratch, bytes) != hipSuccess) {
        result = fail(NH_ENOMEM, "allocation of the tuning scratch failed");
        break;
      }
      hipMemsetAsync(scratch, 0, bytes, e->stream);
      char* c = static_cast<char*>(scratch);
      nh::SweepArgs<double> a64{};
      nh::SweepArgs<float> a32{};
      auto fill = [&](int i, double v) {
        if (e->fp32)
          hipLaunchKernelGGL((nh::k_fill<float>), dim3(nblocks(nk)),
                             dim3(nh::kBlock), 0, e->stream, (long)nk,
                             (float)v, (float*)(c + i * nk * es));
        else
          hipLaunchKernelGGL((nh::k_fill<double>), dim3(nblocks(nk)),
                             dim3(nh::kBlock), 0, e->stream, (long)nk, v,
                             (double*)(c + i * nk * es));
      };
      fill(0, 1.0);
      for (int i = 1; i < 5; ++i) fill(i, 0.25);
      double best = 1e300;
      for (const auto& t : kTiles) {
        if (!tile_ok(t[0], t[1], e->sweep_m)) continue;
        int ntx = (m->grid.nx + 1 + t[0] - 1) / t[0];
        int nty = (m->grid.ny + 1 + t[1] - 1) / t[1];
        if ((long)ntx * nty > 8192) continue;  // scratch measures
        double* pbase = (double*)(c + 6 * nk * es);
        auto setup = [&](auto& s) {
          using TT = typename std::remove_pointer<decltype(s.diag)>::type;
          using U = typename std::remove_const<TT>::type;
          s.ncx = m->grid.nx + 1;
          s.ncy = m->grid.ny + 1;
          s.BX = t[0];
          s.BY = t[1];
          s.ntx = ntx;
          s.ntiles = ntx * nty;
          U* base = (U*)c;
          s.diag = base;
          s.cE = base + nk;
          s.cW = base + 2 * nk;
          s.cN = base + 3 * nk;
          s.cS = base + 4 * nk;
          s.rhs = base + 5 * nk;
          s.p[0] = pbase;
          s.p[1] = pbase + nk;
          s.p[2] = pbase + nk;
          s.omega = m->omega_dev;
          s.nom = (int)m->omega.size();
          s.part = pbase + 2 * nk;
        };
        nh::SweepLaunch Lc{0, 1, 2, 0, nh::kSweepS, 0, 0, nullptr, nullptr, 0};
        float ms_min = 1e30f;
        for (int r = 0; r <= reps; ++r) {
          (void)hipEventRecord(a, e->stream);
          if (e->fp32) {
            setup(a32);
            hipLaunchKernelGGL((nh::k_sweep_tb<float, nh::kSweepB,
                                               nh::kSweepS, nh::kSweepMBig>),
                               dim3(a32.nblocks()), dim3(nh::kSweepB),
                               sweep_lds_bytes(t[0], t[1]), e->stream, a32,
                               Lc);  // FP32 ensembles sweep with 3 points
          } else {
            setup(a64);
            hipLaunchKernelGGL((nh::k_sweep_tb<double, nh::kSweepB,
                                               nh::kSweepS, nh::kSweepM>),
                               dim3(a64.nblocks()), dim3(nh::kSweepB),
                               sweep_lds_bytes(t[0], t[1]), e->stream, a64,
                               Lc);
          }
          (void)hipEventRecord(b, e->stream);
          if (hipEventSynchronize(b) != hipSuccess) {
            result = fail(NH_EDEVICE, "tuning launch failed");
            break;
          }
          float ms = 0.f;
          (void)hipEventElapsedTime(&ms, a, b);
          if (r > 0) ms_min = std::min(ms_min, ms);  // first: warmup
        }
        if (result != NH_OK) break;
        if (ms_min < best) {
          best = ms_min;
          bx = t[0];
          by = t[1];
        }
      }
      hipStreamSynchronize(e->stream);
      hipFree(scratch);
      if (result != NH_OK) break;
      done.push_back({shape, {bx, by}});
    }
    if ((result = set_member_tile(m, bx, by)) != NH_OK) break;
  }
  hipEventDestroy(a);
  hipEventDestroy(b);
  e->dirty = true;
  return result;
}

nh_status nh_ensemble_run(nh_ensemble* e, int64_t nsteps) {
  if (!e) return fail(NH_EINVAL, "null ensemble");
  if (nsteps < 0) return fail(NH_EINVAL, "nsteps < 0");
  if (e->live.empty()) return fail(NH_ESTATE, "no member has a valid state");
  for (int id : e->live)
    if (!(e->mem[id]->st.dt_next > 0))
      return fail(NH_ESTATE, "member " + std::to_string(id) +
                                 ": dt is not positive");
  nh_status st;
  if (e->dirty) {
    st = e->fp32 ? ens_build<float>(e) : ens_build<double>(e);
    if (st != NH_OK) return st;
  }
  if ((st = ens_gather(e, true)) != NH_OK) return st;
  const int64_t kStatusEvery = 64;
  nh_status worst = NH_OK;
  for (int64_t n = 0; n < nsteps; ++n) {
    st = e->fp32 ? ens_step<float>(e) : ens_step<double>(e);
    if (st != NH_OK) {
      (void)ens_sync(e);
      (void)ens_gather(e, false);
      return st;
    }
    if ((n + 1) % kStatusEvery == 0 || n + 1 == nsteps) {
      nh_status ss = ens_sync(e);
      if (ss != NH_OK && worst == NH_OK) worst = ss;
      if (e->live.empty()) break;
      if (e->dirty) {
        // failed members left: rebuild and continue with the rest
        st = e->fp32 ? ens_build<float>(e) : ens_build<double>(e);
        if (st != NH_OK) return st;
        if ((st = ens_gather(e, true)) != NH_OK) return st;
      }
    }
  }
  if ((st = ens_gather(e, false)) != NH_OK) return st;
  HIP_TRY(hipStreamSynchronize(e->stream));
  if (worst != NH_OK) return fail(worst, "a member failed (see its stats)");
  return NH_OK;
}

nh_status nh_ensemble_run_graph(nh_ensemble* e, int64_t nsteps) {
  if (!e) return fail(NH_EINVAL, "null ensemble");
  if (nsteps < 0) return fail(NH_EINVAL, "nsteps < 0");
  if (e->solve_path != 2)
    return fail(NH_EINVAL,
                "graph replay needs one-launch solves (solve_path 2)");
  if (e->prof.on)
    return fail(NH_EINVAL, "graph replay runs without profiling");
  if (e->live.empty()) return fail(NH_ESTATE, "no member has a valid state");
  for (int id : e->live)
    if (!(e->mem[id]->st.dt_next > 0))
      return fail(NH_ESTATE, "member " + std::to_string(id) +
                                 ": dt is not positive");
  nh_status st;
  if (e->dirty) {
    st = e->fp32 ? ens_build<float>(e) : ens_build<double>(e);
    if (st != NH_OK) return st;
  }
  if ((st = ens_gather(e, true)) != NH_OK) return st;
  if (!e->step_graph) {
    // one step as a graph: every launch of ens_step, none of which waits
    // for the host with one-launch solves
    HIP_TRY(hipStreamSynchronize(e->stream));
    HIP_TRY(hipStreamBeginCapture(e->stream, hipStreamCaptureModeThreadLocal));
    e->capturing = true;
    st = e->fp32 ? ens_step<float>(e) : ens_step<double>(e);
    e->capturing = false;
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(e->stream, &g);
    if (st != NH_OK) {
      if (g) hipGraphDestroy(g);
      return st;
    }
    if (ce != hipSuccess || !g)
      return fail(NH_EDEVICE, std::string("step capture: ") +
                                  hipGetErrorString(ce));
    const hipError_t ie =
        hipGraphInstantiate(&e->step_graph, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (ie != hipSuccess) {
      e->step_graph = nullptr;
      return fail(NH_EDEVICE, std::string("step graph: ") +
                                  hipGetErrorString(ie));
    }
  }
  const int64_t kStatusEvery = 64;
  nh_status worst = NH_OK;
  for (int64_t n = 0; n < nsteps; ++n) {
    HIP_TRY(hipGraphLaunch(e->step_graph, e->stream));
    if ((n + 1) % kStatusEvery == 0 || n + 1 == nsteps) {
      nh_status ss = ens_sync(e);
      if (ss != NH_OK && worst == NH_OK) worst = ss;
      if (e->dirty) break;  // a member failed: the tables change
    }
  }
  if ((st = ens_gather(e, false)) != NH_OK) return st;
  HIP_TRY(hipStreamSynchronize(e->stream));
  if (worst != NH_OK) return fail(worst, "a member failed (see its stats)");
  return NH_OK;
}

nh_status nh_ensemble_read_state(nh_ensemble* e, int32_t k, double* h,
                                 double* hu, double* hv, double* w,
                                 double* p) {
  nh_status st = ens_check_member(e, k);
  if (st != NH_OK) return st;
  HIP_TRY(hipStreamSynchronize(e->stream));
  nh::EnsMember rec;
  HIP_TRY(hipMemcpy(&rec, e->dmem + k, sizeof(rec), hipMemcpyDeviceToHost));
  e->mem[k]->pcur = rec.rot;
  return nh_read_state(e->mem[k], h, hu, hv, w, p);
}

nh_status nh_ensemble_get_stats(const nh_ensemble* e, int32_t k,
                                nh_stats* out) {
  nh_status st = ens_check_member(e, k);
  if (st != NH_OK) return st;
  if (!out) return fail(NH_EINVAL, "null argument");
  *out = e->mem[k]->st;
  out->adjoint_sweeps = 0;
  if (e->failed[k]) out->last_status = e->member_status[k];
  return NH_OK;
}

nh_status nh_ensemble_profile(nh_ensemble* e, int32_t on) {
  if (!e) return fail(NH_EINVAL, "null ensemble");
  HIP_TRY(hipStreamSynchronize(e->stream));
  e->prof.flush();
  e->prof.on = on > 0;
  e->prof.sample = on > 1 ? on : 1;
  e->prof.nbatch = 0;
  if (e->prof.on) std::memset(&e->prof.pr, 0, sizeof(e->prof.pr));
  return NH_OK;
}

nh_status nh_ensemble_get_profile(nh_ensemble* e, nh_profile_t* out) {
  if (!e || !out) return fail(NH_EINVAL, "null argument");
  HIP_TRY(hipStreamSynchronize(e->stream));
  e->prof.flush();
  *out = e->prof.pr;
  return NH_OK;
}

void nh_ensemble_destroy(nh_ensemble* e) {
  if (!e) return;
  if (e->stream) hipStreamSynchronize(e->stream);
  for (nh_solver* m : e->mem) nh_destroy(m);
  if (e->table) hipFree(e->table);
  if (e->dmem) hipFree(e->dmem);
  if (e->dmem_live) hipFree(e->dmem_live);
  if (e->slot) hipHostFree(e->slot);
  if (e->psync) hipFree(e->psync);
  if (e->step_graph) hipGraphExecDestroy(e->step_graph);
  e->prof.release();
  if (e->own_stream) hipStreamDestroy(e->stream);
  delete e;
}

}  // extern "C"
