"""Oracle state of the circular dam-break of Section 7.7 (the workload of
Table 2) at t = 1 s.

Runs the oracle (FP64) on n x n cells with the stop tolerance eps of eq. (32)
step by step until t >= 1 s (the last step overshoots by less than one dt, as
the GPU run that stops at the same step count), and writes the lattice of
cells spaced n/125 apart (every cell for n <= 125), the full-field maxima,
the number of steps, t and the sweep counts, to dambreak_{n}_t1.npz.

Calls only the CPU oracle and the seeded input generators.  Usage:
    python tests/golden/make_dambreak_reference.py n [eps]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.oracle import Oracle, Params  # noqa: E402
from paper_1706_04551_amd import inputs  # noqa: E402


def main(n: int, eps: float = 1e-5):
    c = inputs.case_dambreak(n=n, eps=eps)
    o = Oracle(Params(**c.param_dict()))
    o.set_bathymetry(c.H)
    o.set_state(c.h, c.hu, c.hv)
    t0 = time.time()
    steps = 0
    while o.stats()["t"] < 1.0:
        if o.step() != 0:
            raise SystemExit(f"oracle failed at step {steps}")
        steps += 1
        if steps % 50 == 0:
            print(f"step {steps} t={o.stats()['t']:.4f} "
                  f"{time.time() - t0:.0f} s", flush=True)
    r, st = o.state(), o.stats()
    stride = max(1, n // 125)
    out = {q: r[q][::stride, ::stride] for q in ("h", "hu", "hv")}
    out.update({"max_" + q: np.abs(r[q]).max() for q in ("h", "hu", "hv")})
    path = os.path.join(HERE, f"dambreak_{n}_t1.npz")
    np.savez_compressed(path, stride=stride, steps=steps, t=st["t"],
                        sweeps_total=st["sweeps_total"], solves=st["solves"],
                        eps=eps, **out)
    print("wrote", path, steps, st)


if __name__ == "__main__":
    main(int(sys.argv[1]), float(sys.argv[2]) if len(sys.argv) > 2 else 1e-5)
