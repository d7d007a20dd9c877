"""Benchmark: full non-hydrostatic time steps (FV + pressure solve) on one GPU.

Workload (default): the 512 x 512 island basin, FP64 -- seeded bathymetry of
depth 2-20 m with a dry island, Gaussian hump of 0.5 m, walls, CFL 0.7 (the
largest the 2D MUSCL-minmod + Heun stage with the summed CFL form keeps
round-off from growing at), relaxed-Jacobi solve with a 64-sweep
Chebyshev/Leja schedule, tolerance 1e-10 on the plain-Jacobi update size.
Inputs are synthetic (seeded generators).

A step is one full TVD-RK2 step: two finite-volume stages, two pressure
assemblies, two solves and two corrections, plus the CFL reduction.  The
timed region starts from the workload's initial state already resident in
device memory (the warmup runs first and the state is then reset).

Prints one JSON line with the metric, the roofline of the dominant kernel
(the relaxation sweep), the error against stored oracle states of the same
workload (tests/golden, written by scripts that call only the oracle) and the
CPU oracle's rate on a bounded sample, on one core and on every host core.
"""
from __future__ import annotations

import argparse
import json
import re
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E, published
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_solve_kernels.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1706_04551_amd", "csrc", f)
                  for f in ("kernels.hpp", "nhswe.hip")]
COPY_CAL_BYTES = 256 << 20
GOLDEN = os.path.join(ROOT, "tests", "golden")
ALG_BYTES_SWEEP = {"f64": 40, "f32": 20}   # per corner per sweep (matrix-free
                                           # minimum: r p, h, H, rhs; w p)
# Compulsory HBM bytes per corner of one launch of the temporally blocked
# sweep kernel: the five row coefficients and the right-hand side (bulk type)
# and the FP64 iterate read once, the iterate written once.  The launch's
# sweeps run from LDS and registers, so this, not ALG_BYTES_SWEEP x sweeps,
# is what a launch must move.
BLOCKED_BYTES_LAUNCH = {"f64": 64, "f32": 40}
FULL_STEP_BASE = {"f64": 384.0, "f32": 192.0}   # flux, assembly, correction
# Compulsory bytes per cell of one adjoint step outside its transposed
# solves: per stage the derivative kernels' arrays, each read or written once
# (FP32 bulk: flux derivatives 48 + 64, pressure-row cotangents 104 + 92,
# correction 32 + 44, transposed rows 32, scaled max 8, halvings 24, axpy 12 =
# 460 B; FP64: 888 B), both stages, plus the forward stage re-evaluation of
# the step (FULL_STEP_BASE).
ADJ_STEP_BASE = {"f64": 2 * 888.0 + 384.0, "f32": 2 * 460.0 + 192.0}
# One-launch solve (k_solve_persist): per corner and sweep the update reads
# five LDS neighbours and writes one (48 B of LDS traffic) and does 13 FP64
# flops (a product, four fused multiply-adds, a difference, a product with
# the reciprocal diagonal, a fused update).  Its compulsory HBM bytes are
# those of one pass per solve: rows, rhs and iterate read, result written.
PERSIST_FLOPS = 13
PERSIST_LDS_BYTES = 48
FP64_VECTOR_PEAK_TFLOPS = 78.6      # 256 CUs x 128 FP64 flops/clk x 2.4 GHz
LDS_PEAK_GBS = 256 * 128 * 2.4      # 256 CUs x 128 B/clk x 2.4 GHz


# The timed runs time only the back-to-back sweep batch of one relaxation
# cycle in PROFILE_SAMPLE (HIP events on the solver's stream); timing every
# phase stalls the queue at each event pair and costs ~13 % of a step, so the
# phase split comes from a separate run of PHASE_STEPS steps.
PROFILE_SAMPLE = 8
PHASE_STEPS = 100
PHASES = ("fv_ms", "assemble_ms", "solve_ms", "correct_ms")


def phase_split(pr, steps):
    return {"steps": steps, **{k: round(pr[k], 2) for k in PHASES}}


def alg_bytes_per_cell_step(kbar: float, prec: str) -> float:
    """Bytes per cell-step of the per-sweep model: flux stages 56 + 88,
    assembly 2 x 48, corrections 2 x 72, sweeps 2 x Kbar x 40 (FP64), every
    sweep a full pass over memory; FP32 bulk halves every term.  With
    temporal blocking the sweeps move less than this: bytes / time is an
    effective rate that may exceed the HBM peak."""
    b = 384.0 + 80.0 * kbar
    return b if prec == "f64" else b / 2.0


def blocked_bytes_per_cell_step(kbar: float, prec: str,
                                one_launch: bool = False) -> float:
    """Compulsory bytes per cell-step of the design: flux, assembly and
    correction as in the per-sweep model, and per solve Kbar / 8 launches of
    the sweep kernel at BLOCKED_BYTES_LAUNCH per corner (two solves); with
    one-launch solves one such pass per solve."""
    per_solve = 1.0 if one_launch else kbar / 8.0
    return FULL_STEP_BASE[prec] + 2.0 * per_solve * BLOCKED_BYTES_LAUNCH[prec]


def persist_roofline(pr, prec, ncorn, traffic, copy_gbs):
    # traffic: HBM bytes per sweep of the grid from the counter runs, or None
    """Roofline of the one-launch solve kernel from the HIP-event timing of
    its launches (both solves of one step in PROFILE_SAMPLE) and the sweeps
    those launches did (counted on the device): its work runs from registers
    and LDS, so the roof is the FP64 vector rate (13 flops per corner-sweep);
    the LDS rate and the compulsory HBM rate are reported beside it."""
    launches = max(1, pr["solve_kernel_launches"])
    sec = pr["solve_kernel_ms"] * 1e-3 / launches
    sweeps = pr["solve_kernel_sweeps"] / launches
    if traffic:   # bytes per sweep of the grid -> per launch
        traffic = int(traffic * sweeps)
    cs = ncorn * sweeps
    flops = PERSIST_FLOPS * cs
    achieved = flops / sec / 1e12 if sec > 0 else None
    hbm = BLOCKED_BYTES_LAUNCH[prec] * ncorn
    return {"bound": "alu",
            "achieved": round(achieved, 3) if achieved else None,
            "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": (round(achieved / FP64_VECTOR_PEAK_TFLOPS, 4)
                     if achieved else None),
            "traffic": traffic,
            "traffic_frac": (round(traffic / sec / 1e9 / HBM_PEAK_GBS, 4)
                             if traffic and sec > 0 else None),
            "kernel": "k_solve_persist",
            "avg_launch_us": round(sec * 1e6, 3),
            "sweeps_per_launch": round(sweeps, 3),
            "corners_per_launch": int(ncorn),
            "alg_flops_per_launch": int(flops),
            "alg_basis": (f"{PERSIST_FLOPS} FP64 flops per corner per sweep "
                          "(the relaxation update of eq. 32), over the "
                          "sweeps of the launch; the FP64 vector peak"),
            "lds_GBps": round(PERSIST_LDS_BYTES * cs / sec / 1e9, 1),
            "lds_frac": round(PERSIST_LDS_BYTES * cs / sec / 1e9 /
                              LDS_PEAK_GBS, 4),
            "hbm_compulsory_GBps": round(hbm / sec / 1e9, 1),
            "copy_GBps": copy_gbs,
            "timed_launches": f"both solves of 1 step in {PROFILE_SAMPLE}"}


def sweep_roofline(pr, prec, kernel, traffic, copy_gbs):
    """Roofline of the sweep kernel from the HIP-event timing of its
    back-to-back launches: algorithmic bytes = BLOCKED_BYTES_LAUNCH x the
    corners one launch covers; `traffic` (bytes per launch from the counter
    runs, or None) gives the fraction of the peak actually moved."""
    launches = max(1, pr["sweep_kernel_launches"])
    sweep_ms = pr["sweep_kernel_ms"] / launches
    corners = (pr["sweep_kernel_corner_sweeps"] /
               max(1, pr["sweep_kernel_sweeps"]))
    alg = BLOCKED_BYTES_LAUNCH[prec] * corners
    sec = sweep_ms * 1e-3
    achieved = alg / sec / 1e9 if sec > 0 else None
    model = ALG_BYTES_SWEEP[prec] * pr["sweep_kernel_corner_sweeps"] / launches
    return {"bound": "hbm",
            "achieved": round(achieved, 1) if achieved else None,
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
            "traffic": traffic,
            "traffic_frac": (round(traffic / sec / 1e9 / HBM_PEAK_GBS, 4)
                             if traffic and sec > 0 else None),
            "kernel": kernel, "avg_launch_us": round(sweep_ms * 1e3, 3),
            "sweeps_per_launch": round(pr["sweep_kernel_sweeps"] / launches,
                                       3),
            "corners_per_launch": int(round(corners)),
            "alg_bytes_per_launch": int(alg),
            "alg_basis": (f"{BLOCKED_BYTES_LAUNCH[prec]} B per corner per "
                          "launch: 5 coefficients + rhs + iterate read, "
                          "iterate written, once per launch of its sweeps"),
            "per_sweep_model_GBps": (round(model / sec / 1e9, 1)
                                     if sec > 0 else None),
            "copy_GBps": copy_gbs,
            "timed_cycles": f"1 in {PROFILE_SAMPLE}"}


def ens_solve_roofline(pr, prec, stats, corners):
    """Roofline of the one-launch ensemble solve from the HIP-event timing of
    the solves of one step in PROFILE_SAMPLE: the blocked algorithmic bytes
    of its 8-sweep blocks (BLOCKED_BYTES_LAUNCH per corner and block; each
    member's mean sweeps per solve over the run / 8 blocks) over the mean
    solve time.  The sweep launches it replaces are priced the same way."""
    n = max(1, pr["solve_kernel_launches"])
    ms = pr["solve_kernel_ms"] / n
    blocks = sum(c * s["sweeps_total"] / max(1, s["solves"]) / 8.0
                 for c, s in zip(corners, stats))
    alg = BLOCKED_BYTES_LAUNCH[prec] * blocks
    sec = ms * 1e-3
    achieved = alg / sec / 1e9 if sec > 0 else None
    return {"bound": "hbm",
            "achieved": round(achieved, 1) if achieved else None,
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
            "traffic": None, "traffic_frac": None,
            "kernel": "k_ens_solve", "avg_launch_us": round(ms * 1e3, 3),
            "corner_blocks_per_launch": int(round(blocks)),
            "alg_bytes_per_launch": int(alg),
            "alg_basis": (f"{BLOCKED_BYTES_LAUNCH[prec]} B per corner per "
                          "block of 8 sweeps (5 coefficients + rhs + iterate "
                          "read, iterate written), the members' mean sweeps "
                          "per solve"),
            "timed_launches": f"both solves of 1 step in {PROFILE_SAMPLE}"}


def copy_bandwidth():
    """Achievable HBM bandwidth: a 1 GiB device-to-device copy (1 GiB read +
    1 GiB written), best of 5, timed with events on torch's stream."""
    import torch
    n = (1 << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = None
    for _ in range(5):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del a, b
    torch.cuda.empty_cache()
    return round(2 * (1 << 30) / (best * 1e-3) / 1e9, 1)


def golden(name):
    """A stored oracle state (tests/golden), or None if not generated."""
    import numpy as np
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        return None
    return np.load(path)


def lattice_err(g, ref, stride, suffix="", prefix=""):
    """Normwise max difference on the stored lattice: h by the oracle's
    max|h|, the discharges by the larger of max|hu|, max|hv| (full fields)."""
    import numpy as np
    sq = max(float(ref[prefix + "max_hu" + suffix]),
             float(ref[prefix + "max_hv" + suffix]))
    out = {}
    for k, scale in (("h", float(ref[prefix + "max_h" + suffix])), ("hu", sq),
                     ("hv", sq)):
        out[k] = float(np.abs(g[k][::stride, ::stride] -
                              ref[prefix + k + suffix]).max() / scale)
    return out


def storage_drift(ref, sto, suffix="", prefix="", sto_prefix=""):
    """The same measure for the oracle with its state rounded to FP32 after
    every step: what FP32 storage of the state alone changes."""
    import numpy as np
    sq = max(float(ref[prefix + "max_hu" + suffix]),
             float(ref[prefix + "max_hv" + suffix]))
    out = {}
    for k, scale in (("h", float(ref[prefix + "max_h" + suffix])), ("hu", sq),
                     ("hv", sq)):
        out[k] = float(np.abs(sto[sto_prefix + k + suffix] -
                              ref[prefix + k + suffix]).max() / scale)
    return out


def rounded(d, digits=3):
    return {k: (float(f"{v:.{digits}e}") if isinstance(v, float) else v)
            for k, v in d.items()}


def kernel_source_hash() -> str:
    """Hash of the solve kernels' source and of the sweep tile
    configuration."""
    import hashlib
    import re
    with open(KERNEL_SOURCES[0]) as fh:
        k = fh.read()
    a = k.index("constexpr int kSweepB")
    b = k.index("// correction (eq. 26-27")
    c = k.index("// A whole relaxation solve in one launch")
    d = k.index("k_correct(CorrectArgs<T> a)")
    with open(KERNEL_SOURCES[1]) as fh:
        host = fh.read()
    tiles = "".join(re.findall(r"s->tb[xy] = \d+;", host))
    # the code only: comments may change without new counter runs
    code = re.sub(r"//[^\n]*", "", k[a:b] + k[c:d])
    code = re.sub(r"\s+", " ", code)
    return hashlib.sha256((code + tiles).encode()).hexdigest()[:16]


def measured_traffic(workload_name: str, prec: str, kernel="k_sweep_tb"):
    """HBM bytes of the solve kernel from the committed rocprofv3 counter
    runs (FETCH_SIZE + WRITE_SIZE scaled by a plain copy of known size): per
    launch of 8 sweeps, or for the one-launch solve per sweep of the grid
    (its launches differ in their sweep counts); None when the kernel
    sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except OSError:
        return None
    key = f"{workload_name}-{prec}"
    if (t.get("source_sha") != kernel_source_hash() or key not in t or
            t[key].get("kernel", "k_sweep_tb") != kernel):
        return None
    if kernel == "k_solve_persist":
        return t[key]["bytes_per_sweep"]
    return t[key]["bytes_per_launch"]


def copy_calibration():
    """A plain device copy of COPY_CAL_BYTES (read + write of known size),
    run so that the counter runs can scale FETCH_SIZE / WRITE_SIZE."""
    import torch
    a = torch.empty(COPY_CAL_BYTES // 8, dtype=torch.float64, device="cuda")
    a.fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()


# runtimes to t = 1 s of the circular dam-break in the paper's Table 2 (FP64
# CUDA on a GTX Titan Black), by (cells per side, eps of eq. 32)
TABLE2_S = {(250, 1e-3): 0.64, (500, 1e-3): 5.79, (750, 1e-3): 17.33,
            (1000, 1e-3): 40.47, (1250, 1e-3): 79.67, (1500, 1e-3): 136.12,
            (250, 1e-4): 1.88, (500, 1e-4): 8.44, (750, 1e-4): 25.78,
            (1000, 1e-4): 57.23, (1250, 1e-4): 143.19, (1500, 1e-4): 243.86,
            (250, 1e-5): 3.47, (500, 1e-5): 33.54, (750, 1e-5): 99.58,
            (1000, 1e-5): 198.91, (1250, 1e-5): 381.89, (1500, 1e-5): 662.51,
            # the hydrostatic (SWE-only) code of the same table
            (250, "swe"): 0.64, (500, "swe"): 2.29, (750, "swe"): 7.17,
            (1000, "swe"): 16.75, (1250, "swe"): 33.88, (1500, "swe"): 56.38}


def workload(name: str, prec: str, n=None, eps=None):
    from paper_1706_04551_amd import inputs
    if name == "dambreak":
        n, eps = n or 1000, eps or 1e-5
        c = inputs.case_dambreak(n=n, eps=eps, precision=prec)
        return c, (f"circular dam-break {n}x{n} on [-5,5]^2 (Section 7.7), "
                   f"open sides, CFL 0.9, to t = 1 s, {prec.upper()}, "
                   f"Jacobi+SRJ(64) tol={eps:g}")
    if name == "c2":
        n = n or 512
        c = inputs.case_c2(n=n, precision=prec)
        desc = (f"island basin {n}x{n} dx=1m, depth 2-20 m + dry island, "
                f"hump 0.5 m, walls, {prec.upper()}, Jacobi+SRJ(64) "
                f"tol={c.solve_tol:g}")
        return c, desc
    if name == "c3":
        c = inputs.case_c3()
        return c, "plane beach 2048x2048 dx=0.05m, solitary wave A=0.3, breaking, FP32"
    raise SystemExit(f"unknown workload {name}")


def host_cpu():
    """Model name of the host CPU and the cores this process may run on (at
    most 16, the host share of one GPU)."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, min(len(os.sched_getaffinity(0)), 16)


def _oracle_runs(cases, steps: int, copies: int):
    """Wall time of `copies` independent oracle runs of every case for
    `steps` steps at once, one thread each (the oracle's ctypes calls release
    the interpreter lock, so the copies run on separate cores)."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle.oracle import Oracle, Params

    def prepared(c):
        o = Oracle(Params(**c.param_dict()))
        o.set_bathymetry(c.H)
        o.set_state(c.h, c.hu, c.hv)
        return o
    jobs = [prepared(c) for _ in range(copies) for c in cases]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=copies) as ex:
        codes = list(ex.map(lambda o: o.run(steps), jobs))
    wall = time.perf_counter() - t0
    if any(codes):
        return None, None
    st = jobs[0].stats()
    return wall, st["sweeps_total"] / max(1, st["solves"])


def cpu_baseline(cases, steps: int, what: str):
    """The FP64 oracle as it stands on the first `steps` steps of the same
    workload (`cases`: the grid, or the sampled members): once on one core,
    then one copy per host core at once; value = the all-core rate."""
    model, cores = host_cpu()
    cells = sum(c.nx * c.ny for c in cases)
    t1, kbar = _oracle_runs(cases, steps, 1)
    if t1 is None:
        return None
    tn, _ = _oracle_runs(cases, steps, cores)
    if tn is None:
        return None
    one = cells * steps / t1 / 1e6
    alln = cores * cells * steps / tn / 1e6
    return {"value": round(alln, 4), "unit": "Mcell-steps/s", "cores": cores,
            "kind": "oracle",
            "sample": (f"first {steps} steps of {what} ({cells} cells, FP64 "
                       f"oracle, {kbar:.0f} sweeps/solve): one copy per core "
                       f"on {cores} cores at once, {tn:.1f} s wall; one core "
                       f"alone {t1:.1f} s"),
            "single_core_value": round(one, 4), "cpu_model": model}


def ensemble_oracle_err(e, cases, steps):
    """Members sampled two per side against their stored oracle states after
    the workload's 500 steps (tests/golden/c4_members_500.npz): the worst
    member per side, with the FP32-storage drift of the same member."""
    ref = golden("c4_members_500.npz")
    if ref is None or steps != int(ref["steps"]):
        return {"reason": "stored member states not generated for this "
                          "step count"}
    per_side = {}
    for k in (int(m) for m in ref["members"]):
        pre = f"m{k}_"
        st = int(ref[pre + "stride"])
        err = lattice_err(e.state(k), ref, st, prefix=pre)
        drift = storage_drift(ref, ref, prefix=pre, sto_prefix=pre + "sto_")
        side = str(int(ref[pre + "side"]))
        worst = per_side.get(side)
        if worst is None or max(err.values()) > max(worst["err"].values()):
            per_side[side] = {"member": k, "err": rounded(err),
                              "fp32_storage_alone": rounded(drift)}
            if pre + "stoh_h" in ref.files:
                per_side[side]["depth_rounded_to_fp32"] = rounded(
                    storage_drift(ref, ref, prefix=pre,
                                  sto_prefix=pre + "stoh_"))
    return {"steps": steps, "per_side": per_side,
            "reference": ("tests/golden/c4_members_500.npz: the oracle "
                          "(FP64) with each member's configuration, 2 "
                          "members per side, 64 x 64 sampled cells")}


def run_ensemble(args):
    """The 64-scenario ensemble: every member advanced `steps` steps by the
    batched launches, tiles picked by the library's tuner."""
    import torch
    from paper_1706_04551_amd import Ensemble, inputs
    cases = inputs.case_c4(precision=args.precision)
    steps = args.steps if args.steps_given else cases[0].steps
    stream = torch.cuda.current_stream()
    graph = getattr(args, "graph", False)
    e = Ensemble.from_cases(cases, stream=stream.cuda_stream,
                            solve_path=2 if graph else
                            getattr(args, "solve_path", 0))
    e.tune(3)
    run = e.run_graph if graph else e.run
    run(args.warmup)
    for k, c in enumerate(cases):
        e.set_state(k, c.h, c.hu, c.hv)
    if graph:
        run(0)            # captures the step for the new tables
    torch.cuda.synchronize()
    # a graph replays without the timing events of the profile
    e.profile(False if graph else PROFILE_SAMPLE)
    t0 = time.perf_counter()
    run(steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    pr = e.get_profile()
    e.profile(False)
    cells = [c.nx * c.ny for c in cases]
    ncell = sum(cells)
    stats = [e.stats(k) for k in range(len(cases))]
    sweeps = sum(s["sweeps_total"] for s in stats)
    solves = sum(s["solves"] for s in stats)
    kbar = sweeps / max(1, solves)
    full_bytes = sum(n * steps * blocked_bytes_per_cell_step(
        s["sweeps_total"] / max(1, s["solves"]), args.precision)
        for n, s in zip(cells, stats))
    model_bytes = sum(n * steps * alg_bytes_per_cell_step(
        s["sweeps_total"] / max(1, s["solves"]), args.precision)
        for n, s in zip(cells, stats))
    oracle_err = ensemble_oracle_err(e, cases, steps)
    ms_step = elapsed * 1e3 / steps
    value = ncell * steps / elapsed / 1e6
    tiles = {}
    for k, c in enumerate(cases):
        tiles[str(c.nx)] = "x".join(map(str, e.tile(k)))
    nph = min(steps, PHASE_STEPS // 2)
    for k, c in enumerate(cases):
        e.set_state(k, c.h, c.hu, c.hv)
    e.profile(True)
    e.run(nph)
    phases = phase_split(e.get_profile(), nph)
    e.profile(False)
    e.close()
    if graph:
        roof = None       # no timing events inside a graph replay
    elif pr["solve_kernel_launches"] > 0:
        roof = ens_solve_roofline(pr, args.precision, stats,
                                  [(c.nx + 1) * (c.ny + 1) for c in cases])
    else:
        roof = sweep_roofline(pr, args.precision, "k_sweep_tb_batch",
                              measured_traffic("c4", args.precision),
                              getattr(args, "copy_gbs", None))
    cpu = None if args.no_cpu else cpu_baseline(
        cases[:4], 4, "the first 4 scenarios of the ensemble")
    out = {
        "metric": "Mcell-steps/s per full step (flux+pressure solve), % HBM roofline, vs FP64 plain",
        "value": round(value, 3), "unit": "Mcell-steps/s", "n_gpus": 1,
        "steps": steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.precision, "data": "synthetic",
        "config": {"workload": (f"ensemble of {len(cases)} basins (dry island on sides >= 256), sides "
                                f"128-1024 (dx=1m), {ncell} cells, "
                                f"{args.precision.upper()} bulk, Jacobi+SRJ(64) "
                                f"tol={cases[0].solve_tol:g}, tuned tiles"),
                   "cells": ncell, "members": len(cases), "steps": steps,
                   "solve_form": ("one launch per solve, each step replayed "
                                  "from a HIP graph" if graph else
                                  "one cooperative launch per solve"
                                  if getattr(args, "solve_path", 0) == 2
                                  else "launches of 8 sweeps"),
                   "mean_sweeps_per_solve": round(kbar, 2),
                   "members_failed": sum(1 for s in stats if s["status"] != 0),
                   "min_sim_time_s": round(min(s["t"] for s in stats), 3),
                   "full_step_hbm_roofline_frac": round(
                       full_bytes / elapsed / (HBM_PEAK_GBS * 1e9), 4),
                   "full_step_per_sweep_model_GBps": round(
                       model_bytes / elapsed / 1e9, 1),
                   "oracle_err": oracle_err,
                   "tiles": tiles,
                   "phase_ms_profiled_run": phases},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    return out


def adjoint_fp64_err(c, gauges, target, steps, ckpt, r32):
    """The FP32-bulk gradient against the FP64 gradient of the same run
    (same grid, steps, checkpoints; the FP64 kernels equal the differentiable
    oracle to ~1e-13 on the tested grids): normwise max and relative L2
    differences of dJ/deta0 and of dJ/dH at fixed eta0, and of J.  Twice:
    at the workload's initial state (water at rest away from the bump:
    every limiter there sits on its kink, where J has no gradient and each
    precision takes another branch wherever rounding decides it) and at a
    base point off the kinks (a broad seeded 2 cm surface field added)."""
    import numpy as np
    from paper_1706_04551_amd import Solver, inputs

    def diffs(a32, a64):
        out = {"J": float(f"{abs(a32['J'] - a64['J']) / abs(a64['J']):.3e}")}
        for name, a, b in (("dJ_deta0", a32["dh0"], a64["dh0"]),
                           ("dJ_dH", a32["dH"] + a32["dh0"],
                            a64["dH"] + a64["dh0"])):
            out[name] = {
                "max": float(f"{np.abs(a - b).max() / np.abs(b).max():.3e}"),
                "l2": float(f"{np.linalg.norm(a - b) / np.linalg.norm(b):.3e}")}
        return out

    def run(prec, eta, tol):
        cc, _, _, _ = inputs.case_c5(precision=prec)
        s = Solver.from_case(cc)
        s.set_state(cc.H + eta, cc.hu, cc.hv)
        r = s.adjoint(steps, gauges, target, ckpt_every=ckpt, adj_tol=tol)
        s.close()
        return r

    c64, eta0, _, _ = inputs.case_c5(precision="f64")
    out = {"at_rest_base": diffs(r32, run("f64", eta0, 1e-10))}
    xc = inputs.centres(c64.nx, c64.dx)
    rng = np.random.default_rng(91)
    base = eta0 + 0.02 * (inputs.gaussian_field(
        rng, c64.nx, c64.ny, c64.nx * c64.dx, c64.ny * c64.dx, xc, xc, 6) -
        0.5)
    g64 = run("f64", base, 1e-10)
    out["off_kinks_base"] = diffs(run("f32", base, 1e-6), g64)
    # the FP64 gradient's own change under seeded +-5e-8 m of noise in eta0
    # (about one FP32 rounding of the surface): dJ/deta0 is ill-conditioned
    # at that scale wherever the limiters' two slopes nearly tie
    noise = 1e-7 * (np.random.default_rng(7).random(base.shape) - 0.5)
    out["fp64_change_under_5e-8m_noise"] = diffs(run("f64", base + noise,
                                                     1e-10), g64)
    out["reference"] = ("the FP64 adjoint of the same run (solve tolerance "
                        "1e-10, transposed solves 1e-10)")
    return out


def run_adjoint(args):
    """Gradient of the gauge misfit of the 1024^2 basin (fixed dt, 2000
    steps, checkpoints every 100) w.r.t. the initial surface and the
    bathymetry: the forward run, the recomputed segments and the adjoint run,
    all inside the timed region.  The gauge record is a seeded synthetic one
    (inputs.synthetic_gauge_record)."""
    import torch
    from paper_1706_04551_amd import Solver, inputs
    c, eta0, gauges, _ = inputs.case_c5(precision=args.precision)
    steps = args.steps if args.steps_given else c.steps
    target = inputs.synthetic_gauge_record(c, gauges, steps)
    stream = torch.cuda.current_stream()
    s = Solver.from_case(c, stream=stream.cuda_stream)
    ckpt = 100
    if args.warmup > 0:     # sizes the work space, compiles nothing
        s.adjoint(steps, gauges, target, ckpt_every=ckpt, adj_tol=1e-6)
        s.set_state(c.h, c.hu, c.hv)
    torch.cuda.synchronize()
    s.profile(PROFILE_SAMPLE)
    t0 = time.perf_counter()
    r = s.adjoint(steps, gauges, target, ckpt_every=ckpt, adj_tol=1e-6)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    pr = s.get_profile()
    st = s.stats()
    s.profile(False)
    nph = min(steps, 2 * PHASE_STEPS)
    s.set_state(c.h, c.hu, c.hv)
    s.profile(True)
    s.adjoint(nph, gauges, target[:nph], ckpt_every=ckpt, adj_tol=1e-6)
    phases = phase_split(s.get_profile(), nph)
    s.profile(False)
    s.close()
    # compulsory bytes of one gradient step: the forward step twice (the run
    # and the recomputation of its segments), the adjoint's derivative
    # kernels, and its transposed solves (their sweeps counted by the library)
    kbar_f = st["sweeps_total"] / max(1, st["solves"])
    kbar_a = st["adjoint_sweeps"] / max(1, 2 * steps)
    step_bytes = (2.0 * blocked_bytes_per_cell_step(kbar_f, args.precision) +
                  ADJ_STEP_BASE[args.precision] +
                  2.0 * kbar_a / 8.0 * BLOCKED_BYTES_LAUNCH[args.precision])
    grad_err = None
    if args.precision == "f32" and not getattr(args, "no_err", False):
        grad_err = adjoint_fp64_err(c, gauges, target, steps, ckpt, r)
    ncell = c.nx * c.ny
    value = ncell * steps / elapsed / 1e6
    roof = sweep_roofline(pr, args.precision, "k_sweep_tb", None,
                          getattr(args, "copy_gbs", None))
    out = {
        "metric": "Mcell-steps/s per full step (flux+pressure solve), % HBM roofline, vs FP64 plain",
        "value": round(value, 3), "unit": "Mcell-steps/s", "n_gpus": 1,
        "steps": steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed * 1e3 / steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.precision, "data": "synthetic",
        "config": {"workload": (f"gradient of a 16-gauge misfit, basin "
                                f"{c.nx}x{c.ny} dx={c.dx:g}m depth 5-50 m, "
                                f"fixed dt={c.dt_fixed:.4f}s, {steps} steps, "
                                f"checkpoints every {ckpt}, "
                                f"{args.precision.upper()} bulk (forward + "
                                "recomputation + adjoint timed)"),
                   "cells": ncell, "J": r["J"],
                   "err_vs_fp64_gradient": grad_err,
                   "forward_sweeps_per_solve": round(kbar_f, 2),
                   "adjoint_sweeps_per_solve": round(kbar_a, 2),
                   "full_step_hbm_roofline_frac": round(
                       c.nx * c.ny * steps * step_bytes / elapsed /
                       (HBM_PEAK_GBS * 1e9), 4),
                   "full_step_bytes_per_cell": round(step_bytes, 1),
                   "phase_ms_profiled_run": phases},
        "roofline": roof,
        "cpu_baseline": None,
    }
    return out


def single_oracle_err(s, case, args):
    """Error of the workload's full run against the stored oracle state of
    the same configuration (an untimed run from the initial state), or the
    reason there is none."""
    name, prec = args.workload, args.precision
    plain = not (getattr(args, "solve_tol", None) or
                 getattr(args, "hydrostatic", False) or
                 getattr(args, "manning", None) or getattr(args, "zones", None))
    if name == "c2" and plain and case.nx == 512:
        ref = golden(f"c2_512_{prec}_1000.npz")
        if ref is None:
            return {"reason": "stored oracle state not generated"}
        st = int(ref["stride"])
        early = int(ref["early_steps"])
        s.set_state(case.h, case.hu, case.hv)
        s.run(early)
        e_early = lattice_err(s.state(), ref, st, f"_{early}")
        s.run(int(ref["steps"]) - early)
        e = lattice_err(s.state(), ref, st)
        out = {"steps": int(ref["steps"]), **rounded(e),
               f"at_{early}_steps": rounded(e_early),
               "reference": (f"tests/golden/c2_512_{prec}_1000.npz: the "
                             f"oracle (FP64) with this configuration, every "
                             f"{st}th cell"),
               "norm": "max |gpu - oracle| / max |oracle| (discharges by "
                       "the larger of max|hu|, max|hv|)"}
        sto = golden("c2_512_f32storage_1000.npz") if prec == "f32" else None
        if sto is not None:
            out["fp32_storage_alone"] = rounded(storage_drift(ref, sto))
            out[f"fp32_storage_alone_at_{early}_steps"] = rounded(
                storage_drift(ref, sto, f"_{early}"))
        return out
    if name == "dambreak" and plain and prec == "f64":
        ref = golden(f"dambreak_{case.nx}_t1.npz")
        if ref is None or float(ref["eps"]) != case.solve_tol:
            return {"reason": "no stored oracle state for this grid and eps"}
        st = int(ref["stride"])
        s.set_state(case.h, case.hu, case.hv)
        s.run(int(ref["steps"]))
        return {"steps": int(ref["steps"]),
                **rounded(lattice_err(s.state(), ref, st)),
                "reference": (f"tests/golden/dambreak_{case.nx}_t1.npz: the "
                              f"oracle at t = 1 s, every {st}th cell")}
    if name == "c3":
        return c3_oracle_err(s, case, args)
    return {"reason": "no stored oracle state for this variant (its parity "
                      "is tested on smaller grids)"}


def c3_oracle_err(s, case, args):
    """Every row of the beach after its full run against the stored 1D
    oracle run (the data are y-invariant), with the FP32-storage drift."""
    import numpy as np
    ref = golden("c3_beach_4000.npz")
    if ref is None or not case.fixed_dt:
        return {"reason": "stored 1D oracle run not generated"}
    early = int(ref["early_steps"])
    s.set_state(case.h, case.hu, case.hv)
    out = {"steps": int(ref["steps"])}
    for n, sfx in ((early, f"_{early}"), (int(ref["steps"]) - early, "")):
        s.run(n)
        g = s.state()
        e, d = {}, {}
        for k in ("h", "hu"):
            r = ref[k + sfx][None, :]
            scale = float(ref["max_" + k + sfx])
            e[k] = float(np.abs(g[k] - r).max() / scale)
            d[k] = float(np.abs(ref["sto_" + k + sfx] - ref[k + sfx]).max() /
                         scale)
        if sfx:
            out[f"at_{early}_steps"] = rounded(e)
            out[f"fp32_storage_alone_at_{early}_steps"] = rounded(d)
        else:
            out.update(rounded(e))
            out["fp32_storage_alone"] = rounded(d)
    out["reference"] = ("tests/golden/c3_beach_4000.npz: the 1D oracle (the "
                        "data are y-invariant), every row compared")
    return out


def run_single(args):
    """One grid (c2 or c3) for args.steps steps from its initial state."""
    import torch
    from paper_1706_04551_amd import Solver
    case, desc = workload(args.workload, args.precision,
                          getattr(args, "n", None),
                          getattr(args, "solve_tol", None))
    if args.workload == "c3":
        # the fixed dt of the stored 1D oracle run (half the 2D CFL limit of
        # the initial state), so that every row can be checked against it
        ref = golden("c3_beach_4000.npz")
        if ref is not None:
            case.fixed_dt, case.dt_fixed = 1, float(ref["dt"])
            desc += f", fixed dt {case.dt_fixed:.5g} s"
    if getattr(args, "solve_tol", None):
        case.solve_tol = args.solve_tol
        desc = re.sub(r"tol=[0-9.e+-]+", f"tol={case.solve_tol:g}", desc)
        if "tol=" not in desc:
            desc += f", tol={case.solve_tol:g}"
    if getattr(args, "hydrostatic", False):
        case.nh_on = 0
        desc += ", hydrostatic (no pressure step)"
    if getattr(args, "manning", None):
        case.manning = args.manning
        desc += f", Manning n={case.manning:g}"
    stream = torch.cuda.current_stream()
    path = getattr(args, "solve_path", 0)
    s = Solver.from_case(case, stream=stream.cuda_stream, solve_path=path)
    if path == 1:
        desc += ", pressure solves in launches of 8 sweeps"
    zones = getattr(args, "zones", None)
    if zones:
        s.set_relaxation((zones,) * 4)   # absorbing zones on every wall
        desc += f", absorbing zones {zones:g} m"
    ncell = case.nx * case.ny
    t_end = None
    if args.workload == "dambreak" and not getattr(args, "steps_given", False):
        # as many steps as reach t = 1 s (an explicit --steps runs that many)
        t_end, k = 1.0, 0
        while s.stats()["t"] < t_end:
            s.run(1)
            k += 1
        args.steps = k
        s.set_state(case.h, case.hu, case.hv)

    # warmup, then reset to the initial state (uploads are outside the timing)
    s.run(args.warmup)
    s.set_state(case.h, case.hu, case.hv)
    torch.cuda.synchronize()
    s.profile(PROFILE_SAMPLE)
    t0 = time.perf_counter()
    s.run(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = s.stats()
    pr = s.get_profile()
    s.profile(False)
    nph = min(args.steps, PHASE_STEPS)
    s.set_state(case.h, case.hu, case.hv)
    s.profile(True)
    s.run(nph)
    phases = phase_split(s.get_profile(), nph)
    s.profile(False)
    oracle_err = (None if getattr(args, "no_err", False)
                  else single_oracle_err(s, case, args))
    s.close()

    kbar = st["sweeps_total"] / max(1, st["solves"])
    value = ncell * args.steps / elapsed / 1e6
    ms_step = elapsed * 1e3 / args.steps

    # roofline of the dominant kernel: the relaxation solve (one launch per
    # solve where the grid fits the co-resident workgroups, else launches of
    # 8 sweeps)
    one_launch = pr["solve_kernel_launches"] > 0
    wl = (f"dambreak{case.nx}" if args.workload == "dambreak"
          else f"c2_{case.nx}" if args.workload == "c2" and case.nx != 512
          else args.workload)
    if one_launch:
        ncorn = (case.nx + 1) * (case.ny + 1)
        roof = persist_roofline(
            pr, args.precision, ncorn,
            measured_traffic(wl, args.precision, "k_solve_persist"),
            getattr(args, "copy_gbs", None))
    else:
        roof = sweep_roofline(
            pr, args.precision, "k_sweep_tb",
            measured_traffic(wl, args.precision),
            getattr(args, "copy_gbs", None))
    sec_step = ms_step * 1e-3
    step_roof_frac = (blocked_bytes_per_cell_step(kbar, args.precision,
                                                  one_launch) *
                      ncell / sec_step / (HBM_PEAK_GBS * 1e9))
    step_eff_gbs = (alg_bytes_per_cell_step(kbar, args.precision) * ncell /
                    sec_step / 1e9)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline([case], args.cpu_steps, "the same workload")

    return {
        "metric": "Mcell-steps/s per full step (flux+pressure solve), % HBM roofline, vs FP64 plain",
        "value": round(value, 3),
        "unit": "Mcell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": desc, "cells": ncell, "steps": args.steps,
                   "sim_time_s": round(st["t"], 4),
                   "mean_sweeps_per_solve": round(kbar, 2),
                   "full_step_hbm_roofline_frac": round(step_roof_frac, 4),
                   "full_step_per_sweep_model_GBps": round(step_eff_gbs, 1),
                   "phase_ms_profiled_run": phases,
                   "oracle_err": oracle_err,
                   **({} if t_end is None else {
                       "time_to_t_end_s": round(elapsed, 4),
                       "paper_table2_s": TABLE2_S.get(
                           (case.nx, case.solve_tol if case.nh_on else "swe")),
                       "paper_hardware": "GTX Titan Black, FP64 CUDA "
                                         "(context: other hardware)"})},
        "roofline": roof,
        "cpu_baseline": cpu,
    }


def variant_summary(out):
    """The figures of a variant run, for the headline line."""
    cfg = out["config"]
    roof = out["roofline"] or {}   # none for a graph replay (no events)
    return {"workload": cfg["workload"], "value": out["value"],
            "unit": out["unit"], "dtype": out["dtype"], "steps": out["steps"],
            "ms_per_step": out["ms_per_step"],
            "mean_sweeps_per_solve": cfg.get("mean_sweeps_per_solve",
                                             cfg.get("forward_sweeps_per_solve")),
            "full_step_hbm_roofline_frac": cfg.get("full_step_hbm_roofline_frac"),
            "full_step_per_sweep_model_GBps": cfg.get(
                "full_step_per_sweep_model_GBps"),
            "sweep_roofline_frac": roof.get("frac"),
            "sweep_traffic_frac": roof.get("traffic_frac"),
            "sweep_kernel": roof.get("kernel"),
            "sweep_avg_launch_us": roof.get("avg_launch_us"),
            **{k: cfg[k] for k in ("oracle_err", "err_vs_fp64_gradient",
                                   "members_failed", "min_sim_time_s",
                                   "sim_time_s", "time_to_t_end_s",
                                   "paper_table2_s", "paper_hardware",
                                   "solve_form")
               if k in cfg}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--precision", default=None, choices=["f64", "f32"],
                    help="default: f64 for c2 and dambreak, f32 for the c3, "
                         "c4 and c5 workloads")
    ap.add_argument("--cpu-steps", type=int, default=6)
    ap.add_argument("--solve-tol", type=float, default=None,
                    help="override the workload's stop tolerance (eq. 32)")
    ap.add_argument("--manning", type=float, default=None,
                    help="Gauckler-Manning n of the friction law (default 0)")
    ap.add_argument("--hydrostatic", action="store_true",
                    help="shallow water only: no pressure step")
    ap.add_argument("--n", type=int, default=None,
                    help="cells per side of the dam-break workload (1000)")
    ap.add_argument("--zones", type=float, default=None,
                    help="width [m] of absorbing relaxation zones on every "
                         "wall (default none)")
    ap.add_argument("--graph", action="store_true",
                    help="c4: one-launch solves, each step replayed from a "
                         "HIP graph (nh_ensemble_run_graph)")
    ap.add_argument("--solve-path", type=int, default=0, choices=[0, 1, 2],
                    help="launch form of the pressure solve: 0 automatic, 1 "
                         "launches of 8 sweeps, 2 one cooperative launch")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-err", action="store_true",
                    help="skip the runs that measure the error against the "
                         "stored oracle states (for profiler runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain copy of 256 MiB (for counter runs)")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the FP32, beach, ensemble and adjoint runs that "
                         "follow the default workload")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only (the time step of one "
              "grid on one device); --gpus must be 1", file=sys.stderr)
        raise SystemExit(2)

    import torch

    assert torch.cuda.is_available(), "no HIP device visible"
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        copy_calibration()
    args.copy_gbs = copy_bandwidth()
    args.steps_given = args.steps is not None
    if args.precision is None:
        args.precision = ("f64" if args.workload in ("c2", "dambreak")
                          else "f32")
    if args.workload == "c4":
        out = run_ensemble(args)
    elif args.workload == "c5":
        out = run_adjoint(args)
    else:
        if args.steps is None:
            args.steps = 1000
        out = run_single(args)
        if (args.workload == "c2" and args.precision == "f64"
                and not args.no_variants):
            # the FP32-bulk, batched and adjoint forms on the same GPU, each
            # timed on its own workload after the headline run
            import copy
            variants = {}

            def note(msg):
                print(f"bench.py: {msg}", file=sys.stderr, flush=True)
            note(f"headline {out['value']} {out['unit']}; variants follow")
            v = copy.copy(args)
            v.precision, v.no_cpu = "f32", True
            variants["c2_fp32_bulk"] = variant_summary(run_single(v))
            note("c2 FP32 done")
            v = copy.copy(args)
            v.no_cpu, v.solve_tol = True, 1e-5   # the paper's tightest (Table 2)
            variants["c2_fp64_eps1e-5"] = variant_summary(run_single(v))
            note("c2 FP64 at eps 1e-5 done")
            v = copy.copy(args)
            v.no_cpu, v.manning = True, 0.012   # the paper's flume roughness
            variants["c2_fp64_manning"] = variant_summary(run_single(v))
            note("c2 FP64 with friction done")
            v = copy.copy(args)
            v.no_cpu, v.zones = True, 32.0   # ~1.5 wavelengths of the hump
            variants["c2_fp64_absorbing_zones"] = variant_summary(
                run_single(v))
            note("c2 FP64 with absorbing zones done")
            v = copy.copy(args)
            v.no_cpu, v.solve_path = True, 1
            variants["c2_fp64_8sweep_launches"] = variant_summary(
                run_single(v))
            note("c2 FP64 with launches of 8 sweeps done")
            v = copy.copy(args)
            v.workload, v.precision, v.no_cpu, v.no_err = "c2", "f32", True, True
            v.n, v.steps = 4096, 10
            variants["c2_4096_fp32_hbm_calibration"] = variant_summary(
                run_single(v))
            note("c2 geometry at 4096^2 FP32 (out of the MALL) done")
            v = copy.copy(args)
            v.workload, v.no_cpu, v.solve_tol = "dambreak", True, 1e-5
            v.n, v.steps, v.steps_given = 1000, None, False
            variants["dambreak_1000_fp64_eps1e-5"] = variant_summary(
                run_single(v))
            note("dam-break of the paper's Table 2 done")
            v = copy.copy(args)
            v.workload, v.precision, v.no_cpu = "c3", "f32", True
            v.steps = 4000          # the beach workload's full run
            variants["c3_beach_fp32"] = variant_summary(run_single(v))
            note("c3 beach done")
            v = copy.copy(args)
            v.workload, v.precision, v.no_cpu = "c4", "f32", True
            v.steps, v.steps_given = None, False
            variants["c4_ensemble_fp32"] = variant_summary(run_ensemble(v))
            note("c4 ensemble done")
            # the same workload with each solve one persistent launch over
            # all members and each step replayed from a HIP graph
            v = copy.copy(args)
            v.workload, v.precision, v.no_cpu = "c4", "f32", True
            v.steps, v.steps_given, v.graph = None, False, True
            variants["c4_ensemble_fp32_one_launch_graph"] = variant_summary(
                run_ensemble(v))
            note("c4 ensemble (graph) done")
            v = copy.copy(args)
            v.workload, v.precision, v.no_cpu, v.warmup = "c5", "f32", True, 0
            v.steps, v.steps_given = None, False
            variants["c5_adjoint_fp32"] = variant_summary(run_adjoint(v))
            out["variants"] = variants
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
