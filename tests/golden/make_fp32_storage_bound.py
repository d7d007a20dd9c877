"""Error that FP32 storage of the state alone causes on the island-free basin.

Runs the oracle (FP64 arithmetic) with the FP32-bulk configuration of the
island-free 512 x 512 basin, rounding h, hu, hv and w to single precision
after every step, and writes the same lattice of sampled cells as
make_c2_reference.py (after 250 and 1000 steps).  Against the unrounded
oracle run this measures how far any computation that stores its state in
FP32 drifts on this workload; the FP32 parity test bounds the GPU by it.

Calls only the CPU oracle and the seeded input generators.  Usage:
    python tests/golden/make_fp32_storage_bound.py
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

STRIDE = 4
EARLY = 250


def f32(a):
    return a.astype(np.float32).astype(np.float64)


def main():
    c = inputs.case_c2(precision="f32", island=False)
    o = Oracle(Params(**c.param_dict()))
    o.set_bathymetry(c.H)
    o.set_state(c.h, c.hu, c.hv)
    t0 = time.time()
    out = {}
    for s in range(c.steps):
        if o.step() != 0:
            raise SystemExit(f"oracle failed at step {s}")
        r = o.state()
        o.set_state(f32(r["h"]), f32(r["hu"]), f32(r["hv"]), f32(r["w"]),
                    r["p"])
        if s + 1 in (EARLY, c.steps):
            sfx = "" if s + 1 == c.steps else f"_{EARLY}"
            r = o.state()
            for k in ("h", "hu", "hv"):
                out[k + sfx] = r[k][::STRIDE, ::STRIDE]
        if (s + 1) % 100 == 0:
            print(f"step {s + 1}  {time.time() - t0:.0f} s", flush=True)
    path = os.path.join(HERE, f"c2wet_512_f32storage_{c.steps}.npz")
    np.savez_compressed(path, stride=STRIDE, early_steps=EARLY, **out)
    print("wrote", path)


if __name__ == "__main__":
    main()
