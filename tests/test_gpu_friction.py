"""Manning friction on the GPU: parity with the FP64 oracle (whose friction is
pinned to the exact decay of the friction law), per-member friction in
ensembles, and the solver's refusal of a negative coefficient.

Tolerances as for the other parity tests: normwise max relative difference
per field <= 1e-9 in FP64 and <= 1e-4 in FP32 bulk mode.  The friction factor
takes a cube root, which the host and device libraries may round differently
in the last bit, so FP64 is compared to the tolerance, not bitwise.  Each case
also checks that friction changes the answer by far more than the tolerance.
"""
import sys

import numpy as np
import pytest

from oracle.oracle import Oracle, Params
from paper_1706_04551_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-9, 1e-4


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def normwise(g, r, k):
    scale = np.abs(r[k]).max()
    if k in ("hu", "hv"):
        scale = max(np.abs(r["hu"]).max(), np.abs(r["hv"]).max())
    return float(np.abs(g[k] - r[k]).max() / max(scale, 1e-300))


def oracle_state(case, steps):
    o = Oracle(Params(**case.param_dict()))
    o.set_bathymetry(case.H)
    o.set_state(case.h, case.hu, case.hv)
    assert o.run(steps) == 0
    return o.state()


def gpu_state(case, steps):
    from paper_1706_04551_amd import Solver
    s = Solver.from_case(case)
    s.run(steps)
    out = s.state()
    s.close()
    return out


def check(case, steps, tol, fields):
    say(f"[case] {case.name} {case.nx}x{case.ny} prec={case.precision} "
        f"manning={case.manning} steps={steps}")
    g = gpu_state(case, steps)
    r = oracle_state(case, steps)
    n = case.manning
    case.manning = 0.0
    r0 = oracle_state(case, steps)
    case.manning = n
    errs = {}
    for k in fields:
        e = errs[k] = normwise(g, r, k)
        say(f"  {k}: max rel diff {e:.3e}; friction changes it by "
            f"{normwise(r0, r, k):.3e}")
        assert e <= tol, (k, e)
    # friction moves hu by ~1e-3 on these cases, far more than the tolerance
    # and than the GPU's distance from the oracle: a path that ignored it
    # would fail
    eff = normwise(r0, r, "hu")
    assert eff > tol and eff > 10 * errs["hu"], (eff, errs["hu"])


@pytest.mark.parametrize("precision,tol", [("f64", TOL64), ("f32", TOL32)])
def test_friction_island_basin_matches_the_oracle(precision, tol):
    c = I.case_c2(n=160, precision=precision)
    c.manning = 0.05
    check(c, 40, tol, ("h", "hu", "hv", "w", "p"))


def test_friction_channel_matches_the_oracle():
    c = I.case_c1()
    c.manning = 0.03
    check(c, 200, TOL64, ("h", "hu", "w", "p"))


def test_ensemble_members_with_their_own_friction():
    from paper_1706_04551_amd import Ensemble
    cases = [I.case_c4_member(k, sides=(n,), precision="f64", island=True)
             for k, n in enumerate((64, 80, 72))]
    for c, n in zip(cases, (0.0, 0.03, 0.06)):
        c.manning = n
    steps = 10
    e = Ensemble.from_cases(cases)
    e.run(steps)
    for k, c in enumerate(cases):
        r = gpu_state(c, steps)
        g = e.state(k)
        for f in ("h", "hu", "hv", "w", "p"):
            assert np.array_equal(g[f], r[f]), (k, f)
    e.close()


def test_negative_or_infinite_friction_is_rejected():
    from paper_1706_04551_amd import NhError, Solver
    for n in (-0.01, float("inf"), float("nan")):
        with pytest.raises(NhError):
            Solver(16, 16, 1.0, 1.0, manning=n)
