"""Error that FP32 storage of the state alone causes on the 512 x 512 basin.

Runs the oracle (FP64 arithmetic) with the FP32-bulk configuration of the
512 x 512 basin, rounding the state after every step to what an FP32-bulk
grid stores -- h - max(H, 0) (the surface elevation over water, the depth
on land), hu, hv and w in single precision (a dry cell stays dry) -- and writes the same lattice of sampled
cells as make_c2_reference.py (after 250 and 1000 steps).  Against the
unrounded oracle run this measures how far any computation that stores its
state in FP32 drifts on this workload; the FP32 parity tests bound the GPU by
it.

Calls only the CPU oracle and the seeded input generators.  Usage:
    python tests/golden/make_fp32_storage_bound.py [island|wet]
"island" (the workload as stated, with the dry island and its wet-dry
front) writes c2_512_f32storage_1000.npz; "wet" (the default, the same basin
without the island) writes c2wet_512_f32storage_1000.npz.
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


def stored_depth(h, H):
    """The depth after FP32 storage of s = h - max(H, 0) (the surface
    elevation over water, the depth on land; dry cells stay dry)."""
    R = np.maximum(H, 0.0)
    d = np.maximum(f32(h - R) + R, 0.0)
    d[h <= 0.0] = 0.0
    return d


def main(island: bool = False):
    c = inputs.case_c2(precision="f32", island=island)
    o = Oracle(Params(**c.param_dict()))
    o.set_bathymetry(c.H)
    o.set_state(c.h, c.hu, c.hv)
    t0 = time.time()
    out = {}
    for s in range(c.steps):
        if o.step() != 0:
            raise SystemExit(f"oracle failed at step {s}")
        r = o.state()
        o.set_state(stored_depth(r["h"], c.H), f32(r["hu"]), f32(r["hv"]),
                    f32(r["w"]), r["p"])
        if s + 1 in (EARLY, c.steps):
            sfx = "" if s + 1 == c.steps else f"_{EARLY}"
            r = o.state()
            for k in ("h", "hu", "hv"):
                out[k + sfx] = r[k][::STRIDE, ::STRIDE]
        if (s + 1) % 100 == 0:
            print(f"step {s + 1}  {time.time() - t0:.0f} s", flush=True)
    tag = "c2" if island else "c2wet"
    path = os.path.join(HERE, f"{tag}_512_f32storage_{c.steps}.npz")
    np.savez_compressed(path, stride=STRIDE, early_steps=EARLY, **out)
    print("wrote", path)


if __name__ == "__main__":
    main(len(sys.argv) > 1 and sys.argv[1] == "island")
