"""Write SHA-256 digests of the oracle's whole state (every cell and corner
of h, hu, hv, w, p, FP64) after 250 and 1000 steps of the island basin
(512 x 512, FP64), so that a GPU run can be compared with it on every value
at the full size, not only on a lattice of sampled cells.

Calls only the CPU oracle and the seeded input generators.  Usage:
    python tests/golden/make_c2_digest.py
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.oracle import Oracle, Params  # noqa: E402
from paper_1706_04551_amd import inputs  # noqa: E402

FIELDS = ("h", "hu", "hv", "w", "p")
SNAPSHOTS = (250, 1000)


def digest(a) -> str:
    """SHA-256 of the array's FP64 values, row-major, little-endian."""
    return hashlib.sha256(
        np.ascontiguousarray(a, dtype="<f8").tobytes()).hexdigest()


def main():
    c = inputs.case_c2(precision="f64")
    o = Oracle(Params(**c.param_dict()))
    o.set_bathymetry(c.H)
    o.set_state(c.h, c.hu, c.hv)
    t0 = time.time()
    out = {"workload": "island basin 512x512 FP64 (inputs.case_c2)",
           "steps": list(SNAPSHOTS), "sha256": {}, "t": {}}
    for s in range(max(SNAPSHOTS)):
        st = o.step()
        if st != 0:
            raise SystemExit(f"oracle status {st} at step {s}")
        if s + 1 in SNAPSHOTS:
            r = o.state()
            out["sha256"][str(s + 1)] = {k: digest(r[k]) for k in FIELDS}
            out["t"][str(s + 1)] = o.stats()["t"]
        if (s + 1) % 100 == 0:
            print(f"step {s + 1}  {time.time() - t0:.0f} s", flush=True)
    path = os.path.join(HERE, "c2_512_f64_digests.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
