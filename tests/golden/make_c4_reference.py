"""Oracle states of ensemble members after the ensemble's full 500 steps.

For two members of every side of the 64-scenario ensemble (the first two of
each side in member order), runs the oracle (FP64 arithmetic) with the
member's FP32-bulk configuration for the 500 steps of the workload, a second
time with its state rounded after every step to what an FP32-bulk grid
stores (h - max(H, 0), hu, hv, w in single precision; the drift that FP32
storage of the state alone causes), and a third time with the depth itself
rounded to single precision after every step (a perturbation of ulp(h) per
step, the size of the rounding of h = s + max(H, 0) that the FP32 kernels
form in every stencil).  Writes, per member, the lattice of
64 x 64 cells spaced side/64 apart, the full-field maxima, t and the sweep
counts, to c4_members_500.npz.

Calls only the CPU oracle and the seeded input generators.  Usage:
    python tests/golden/make_c4_reference.py [workers] [sto|stoh]
(sto or stoh: keep what is stored and redo only the runs of that kind).
"""
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.oracle import Oracle, Params  # noqa: E402
from paper_1706_04551_amd import inputs  # noqa: E402

PER_SIDE = 2
SAMPLES = 64


def members():
    """(member index, side) of the first PER_SIDE members of every side."""
    out, seen = [], {}
    for k in range(64):
        c = inputs.case_c4_member(k)
        if seen.get(c.nx, 0) < PER_SIDE:
            seen[c.nx] = seen.get(c.nx, 0) + 1
            out.append(k)
    return out


def f32(a):
    return a.astype(np.float32).astype(np.float64)


def stored_depth(h, H):
    """The depth after FP32 storage of s = h - max(H, 0) (the surface
    elevation over water, the depth on land; dry cells stay dry)."""
    R = np.maximum(H, 0.0)
    d = np.maximum(f32(h - R) + R, 0.0)
    d[h <= 0.0] = 0.0
    return d


def run(job):
    k, rounded = job     # rounded: False, "sto" or "stoh"
    c = inputs.case_c4_member(k)
    o = Oracle(Params(**c.param_dict()))
    o.set_bathymetry(c.H)
    o.set_state(c.h, c.hu, c.hv)
    t0 = time.time()
    if rounded:
        for s in range(c.steps):
            if o.step() != 0:
                raise SystemExit(f"member {k}: oracle failed at step {s}")
            r = o.state()
            h = (stored_depth(r["h"], c.H) if rounded == "sto"
                 else f32(r["h"]))
            o.set_state(h, f32(r["hu"]), f32(r["hv"]), f32(r["w"]), r["p"])
    elif o.run(c.steps) != 0:
        raise SystemExit(f"member {k}: oracle failed")
    r = o.state()
    st = o.stats()
    stride = c.nx // SAMPLES
    pre = f"m{k}_" + (f"{rounded}_" if rounded else "")
    out = {pre + q: r[q][::stride, ::stride] for q in ("h", "hu", "hv")}
    if not rounded:
        out.update({pre + "max_" + q: np.abs(r[q]).max()
                    for q in ("h", "hu", "hv")})
        out.update({pre + "t": st["t"], pre + "sweeps_total": st["sweeps_total"],
                    pre + "solves": st["solves"], pre + "stride": stride,
                    pre + "side": c.nx})
    print(f"member {k} ({c.nx}^2){' ' + rounded if rounded else ''}: "
          f"{time.time() - t0:.0f} s", flush=True)
    return out


def main(workers: int = 6, only: str = ""):
    ks = members()
    modes = (only,) if only else (False, "sto", "stoh")
    jobs = sorted([(k, r) for k in ks for r in modes],
                  key=lambda j: -inputs.case_c4_member(j[0]).nx)
    out = {"members": np.array(ks), "steps": 500}
    path = os.path.join(HERE, "c4_members_500.npz")
    if only:   # keep what is stored, redo the runs of one kind
        old = np.load(path)
        out.update({k: old[k] for k in old.files if f"_{only}_" not in k})
    with Pool(workers) as p:
        for d in p.imap_unordered(run, jobs):
            out.update(d)
    np.savez_compressed(path, **out)
    print("wrote", path)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 6,
         sys.argv[2] if len(sys.argv) > 2 else "")
