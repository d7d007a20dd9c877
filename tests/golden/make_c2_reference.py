"""Write the oracle's state after the full island-basin run (512 x 512,
1000 steps, and a snapshot after 250 steps) at a lattice of sampled cells,
for the full-size GPU parity tests.

Calls only the CPU oracle and the seeded input generators.  Usage:
    python tests/golden/make_c2_reference.py [f64|f32] [wet]
"wet" selects the same basin without the island.
The FP32 variant runs the oracle (FP64) with the FP32-bulk configuration of
the workload (dry threshold and solver tolerance), which the GPU's FP32 run
is compared against.
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
EARLY = 250     # a second snapshot of the same run


def main(prec: str = "f64", wet: bool = False):
    c = inputs.case_c2(precision=prec, island=not wet)
    o = Oracle(Params(**c.param_dict()))
    o.set_bathymetry(c.H)
    o.set_state(c.h, c.hu, c.hv)
    t0 = time.time()
    early = {}
    for s in range(c.steps):
        st = o.step()
        if st != 0:
            raise SystemExit(f"oracle status {st} at step {s}")
        if s + 1 == EARLY:
            e = o.state()
            early = {f"{k}_{EARLY}": e[k][::STRIDE, ::STRIDE]
                     for k in ("h", "hu", "hv")}
            early.update({f"max_{k}_{EARLY}": np.abs(e[k]).max()
                          for k in ("h", "hu", "hv")})
        if (s + 1) % 100 == 0:
            print(f"step {s + 1}  {time.time() - t0:.0f} s", flush=True)
    r = o.state()
    stats = o.stats()
    tag = "c2wet" if wet else "c2"
    out = os.path.join(HERE, f"{tag}_512_{prec}_{c.steps}.npz")
    np.savez_compressed(
        out, stride=STRIDE, steps=c.steps,
        h=r["h"][::STRIDE, ::STRIDE], hu=r["hu"][::STRIDE, ::STRIDE],
        hv=r["hv"][::STRIDE, ::STRIDE],
        max_h=np.abs(r["h"]).max(), max_hu=np.abs(r["hu"]).max(),
        max_hv=np.abs(r["hv"]).max(), t=stats["t"],
        sweeps_total=stats["sweeps_total"], solves=stats["solves"],
        clamped=stats["clamped"], mass=np.sum(r["h"]), early_steps=EARLY,
        **early)
    print("wrote", out, stats)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "f64",
         len(sys.argv) > 2 and sys.argv[2] == "wet")
