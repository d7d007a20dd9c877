"""Benchmark: full non-hydrostatic time steps (FV + pressure solve) on one GPU.

Workload (default): the 512 x 512 island basin, FP64 -- seeded bathymetry of
depth 2-20 m with a dry island, Gaussian hump of 0.5 m, walls, CFL 0.9,
relaxed-Jacobi solve with a 64-sweep Chebyshev/Leja schedule, tolerance 1e-10
on the plain-Jacobi update size.  Inputs are synthetic (seeded generators).

A step is one full TVD-RK2 step: two finite-volume stages, two pressure
assemblies, two solves and two corrections, plus the CFL reduction.  The
timed region starts from the workload's initial state already resident in
device memory (the warmup runs first and the state is then reset).

Prints one JSON line with the metric, the roofline of the dominant kernel
(the relaxation sweep) and the CPU oracle's rate on a bounded sample.
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_sweep_tb.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1706_04551_amd", "csrc", f)
                  for f in ("kernels.hpp", "nhswe.hip")]
COPY_CAL_BYTES = 256 << 20
ALG_BYTES_SWEEP = {"f64": 40, "f32": 20}   # per corner per sweep (matrix-free
                                           # minimum: r p, h, H, rhs; w p)


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
    """Compulsory bytes per cell-step with ideal stencil reuse:
    flux stages 56 + 88, assembly 2 x 48, corrections 2 x 72, sweeps
    2 x Kbar x 40 (FP64); FP32 bulk halves every term."""
    b = 384.0 + 80.0 * kbar
    return b if prec == "f64" else b / 2.0


def kernel_source_hash() -> str:
    """Hash of the sweep kernel's source and of its tile configuration."""
    import hashlib
    import re
    with open(KERNEL_SOURCES[0]) as fh:
        k = fh.read()
    a = k.index("constexpr int kSweepB")
    b = k.index("// correction (eq. 26-27")
    with open(KERNEL_SOURCES[1]) as fh:
        host = fh.read()
    tiles = "".join(re.findall(r"s->tb[xy] = \d+;", host))
    return hashlib.sha256((k[a:b] + tiles).encode()).hexdigest()[:16]


def measured_traffic(workload_name: str, prec: str):
    """HBM bytes per sweep launch from the committed rocprofv3 counter runs
    (FETCH_SIZE + WRITE_SIZE scaled by a plain copy of known size), or None
    when the kernel sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except OSError:
        return None
    key = f"{workload_name}-{prec}"
    if t.get("source_sha") != kernel_source_hash() or key not in t:
        return None
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
        c = inputs.case_c2(precision=prec)
        desc = (f"island basin 512x512 dx=1m, depth 2-20 m + dry island, "
                f"hump 0.5 m, walls, {prec.upper()}, Jacobi+SRJ(64) "
                f"tol={c.solve_tol:g}")
        return c, desc
    if name == "c3":
        c = inputs.case_c3()
        return c, "plane beach 2048x2048 dx=0.05m, solitary wave A=0.3, breaking, FP32"
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(case, steps: int):
    """The FP64 oracle as it stands, single-threaded, on the first `steps`
    steps of the same workload."""
    from oracle.oracle import Oracle, Params
    kw = case.param_dict()
    o = Oracle(Params(**kw))
    o.set_bathymetry(case.H)
    o.set_state(case.h, case.hu, case.hv)
    t0 = time.perf_counter()
    st = o.run(steps)
    t = time.perf_counter() - t0
    if st != 0:
        return None
    s = o.stats()
    value = case.nx * case.ny * steps / t / 1e6
    return {"value": round(value, 4), "unit": "Mcell-steps/s", "cores": 1,
            "kind": "oracle",
            "sample": (f"first {steps} steps of the same workload "
                       f"({case.nx}x{case.ny}, FP64 oracle, "
                       f"{s['sweeps_total'] / max(1, s['solves']):.0f} sweeps/solve), "
                       f"{t:.1f} s")}


def ensemble_cpu_baseline(cases, members: int, steps: int):
    """The FP64 oracle as it stands, single-threaded, on the first `steps`
    steps of the first `members` scenarios of the ensemble."""
    from oracle.oracle import Oracle, Params
    t = 0.0
    cells = 0
    for c in cases[:members]:
        o = Oracle(Params(**c.param_dict()))
        o.set_bathymetry(c.H)
        o.set_state(c.h, c.hu, c.hv)
        t0 = time.perf_counter()
        if o.run(steps) != 0:
            return None
        t += time.perf_counter() - t0
        cells += c.nx * c.ny
    return {"value": round(cells * steps / t / 1e6, 4), "unit": "Mcell-steps/s",
            "cores": 1, "kind": "oracle",
            "sample": (f"first {steps} steps of the first {members} scenarios "
                       f"({cells} cells, FP64 oracle with the scenarios' "
                       f"tolerance), {t:.1f} s")}


def run_ensemble(args):
    """The 64-scenario ensemble: every member advanced `steps` steps by the
    batched launches, tiles picked by the library's tuner."""
    import torch
    from paper_1706_04551_amd import Ensemble, inputs
    cases = inputs.case_c4(precision=args.precision)
    steps = args.steps if args.steps_given else cases[0].steps
    stream = torch.cuda.current_stream()
    e = Ensemble.from_cases(cases, stream=stream.cuda_stream)
    e.tune(3)
    e.run(args.warmup)
    for k, c in enumerate(cases):
        e.set_state(k, c.h, c.hu, c.hv)
    torch.cuda.synchronize()
    e.profile(PROFILE_SAMPLE)
    t0 = time.perf_counter()
    e.run(steps)
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
    full_bytes = sum(n * steps * alg_bytes_per_cell_step(
        s["sweeps_total"] / max(1, s["solves"]), args.precision)
        for n, s in zip(cells, stats))
    ms_step = elapsed * 1e3 / steps
    value = ncell * steps / elapsed / 1e6
    sweep_ms = pr["sweep_kernel_ms"] / max(1, pr["sweep_kernel_launches"])
    alg = (ALG_BYTES_SWEEP[args.precision] * pr["sweep_kernel_corner_sweeps"]
           / max(1, pr["sweep_kernel_launches"]))
    achieved = alg / (sweep_ms * 1e-3) / 1e9 if sweep_ms > 0 else None
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
    roof = {"bound": "hbm", "achieved": round(achieved, 1) if achieved else None,
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
            "traffic": measured_traffic("c4", args.precision),
            "kernel": "k_sweep_tb_batch",
            "avg_launch_us": round(sweep_ms * 1e3, 3),
            "alg_bytes_per_launch": int(alg),
            "timed_cycles": f"1 in {PROFILE_SAMPLE}"}
    cpu = None if args.no_cpu else ensemble_cpu_baseline(cases, 4, 4)
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
                   "mean_sweeps_per_solve": round(kbar, 2),
                   "members_failed": sum(1 for s in stats if s["status"] != 0),
                   "min_sim_time_s": round(min(s["t"] for s in stats), 3),
                   "full_step_hbm_roofline_frac": round(
                       full_bytes / elapsed / (HBM_PEAK_GBS * 1e9), 4),
                   "tiles": tiles,
                   "phase_ms_profiled_run": phases},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
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
    ncell = c.nx * c.ny
    ncorn = (c.nx + 1) * (c.ny + 1)
    value = ncell * steps / elapsed / 1e6
    sweep_ms = pr["sweep_kernel_ms"] / max(1, pr["sweep_kernel_launches"])
    alg = (ALG_BYTES_SWEEP[args.precision] * pr["sweep_kernel_corner_sweeps"]
           / max(1, pr["sweep_kernel_launches"]))
    achieved = alg / (sweep_ms * 1e-3) / 1e9 if sweep_ms > 0 else None
    roof = {"bound": "hbm", "achieved": round(achieved, 1) if achieved else None,
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
            "traffic": None, "kernel": "k_sweep_tb",
            "avg_launch_us": round(sweep_ms * 1e3, 3),
            "alg_bytes_per_launch": int(alg),
            "timed_cycles": f"1 in {PROFILE_SAMPLE}"}
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
                   "forward_sweeps_per_solve": round(
                       st["sweeps_total"] / max(1, st["solves"]), 2),
                   "phase_ms_profiled_run": phases},
        "roofline": roof,
        "cpu_baseline": None,
    }
    del ncorn
    return out


def run_single(args):
    """One grid (c2 or c3) for args.steps steps from its initial state."""
    import torch
    from paper_1706_04551_amd import Solver
    case, desc = workload(args.workload, args.precision,
                          getattr(args, "n", None),
                          getattr(args, "solve_tol", None))
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
    s = Solver.from_case(case, stream=stream.cuda_stream)
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
    s.close()

    kbar = st["sweeps_total"] / max(1, st["solves"])
    value = ncell * args.steps / elapsed / 1e6
    ms_step = elapsed * 1e3 / args.steps

    # roofline of the dominant kernel: the relaxation sweep
    sweep_ms = pr["sweep_kernel_ms"] / max(1, pr["sweep_kernel_launches"])
    sweeps_per_launch = pr["sweep_kernel_sweeps"] / max(1, pr["sweep_kernel_launches"])
    alg = (ALG_BYTES_SWEEP[args.precision] * pr["sweep_kernel_corner_sweeps"]
           / max(1, pr["sweep_kernel_launches"]))
    achieved = alg / (sweep_ms * 1e-3) / 1e9 if sweep_ms > 0 else None
    roof = {"bound": "hbm", "achieved": round(achieved, 1) if achieved else None,
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
            "traffic": measured_traffic(
                f"dambreak{case.nx}" if args.workload == "dambreak"
                else args.workload, args.precision),
            "kernel": "k_sweep_tb", "avg_launch_us": round(sweep_ms * 1e3, 3),
            "sweeps_per_launch": round(sweeps_per_launch, 3),
            "alg_bytes_per_launch": int(alg),
            "timed_cycles": f"1 in {PROFILE_SAMPLE}"}
    full_step_bytes = alg_bytes_per_cell_step(kbar, args.precision) * ncell
    step_roof_frac = full_step_bytes / (ms_step * 1e-3) / (HBM_PEAK_GBS * 1e9)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(case, args.cpu_steps)

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
                   "phase_ms_profiled_run": phases,
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
    return {"workload": cfg["workload"], "value": out["value"],
            "unit": out["unit"], "dtype": out["dtype"], "steps": out["steps"],
            "ms_per_step": out["ms_per_step"],
            "mean_sweeps_per_solve": cfg.get("mean_sweeps_per_solve",
                                             cfg.get("forward_sweeps_per_solve")),
            "full_step_hbm_roofline_frac": cfg.get("full_step_hbm_roofline_frac"),
            "sweep_roofline_frac": out["roofline"]["frac"],
            "sweep_kernel": out["roofline"]["kernel"],
            **{k: cfg[k] for k in ("members_failed", "min_sim_time_s",
                                   "sim_time_s", "time_to_t_end_s",
                                   "paper_table2_s", "paper_hardware")
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
    ap.add_argument("--cpu-steps", type=int, default=12)
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
    ap.add_argument("--no-cpu", action="store_true")
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
            v = copy.copy(args)
            v.workload, v.precision, v.no_cpu, v.warmup = "c5", "f32", True, 0
            v.steps, v.steps_given = None, False
            variants["c5_adjoint_fp32"] = variant_summary(run_adjoint(v))
            out["variants"] = variants
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
