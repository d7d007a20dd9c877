"""Generation/absorption zones on the GPU against the FP64 oracle (whose zones
are pinned by the absorption of the channel's reflected solitary wave and by
invariants), element by element, and the entry point's argument checks.

Tolerances as for the other parity tests: normwise max relative difference
per field <= 1e-9 in FP64 (the basin with zones on every wall is equal to
the bit) and <= 1e-4 on h and the discharges in FP32 bulk mode.
"""
import sys

import numpy as np
import pytest

from oracle.oracle import Oracle, Params
from paper_1706_04551_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-9, 1e-4
FIELDS = ("h", "hu", "hv", "w", "p")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def normwise(g, r, k):
    scale = np.abs(r[k]).max()
    if k in ("hu", "hv"):
        scale = max(np.abs(r["hu"]).max(), np.abs(r["hv"]).max())
    return float(np.abs(g[k] - r[k]).max() / max(scale, 1e-300))


def both(case, steps, widths, **targets):
    from paper_1706_04551_amd import Solver
    say(f"[case] {case.name} {case.nx}x{case.ny} prec={case.precision} "
        f"zones={widths} steps={steps}")
    s = Solver.from_case(case)
    s.set_relaxation(widths, **targets)
    s.run(steps)
    g = s.state()
    s.close()
    o = Oracle(Params(**case.param_dict()))
    o.set_bathymetry(case.H)
    o.set_state(case.h, case.hu, case.hv)
    o.set_relaxation(widths, **targets)
    assert o.run(steps) == 0
    return g, o.state()


def check(g, r, tol, fields=FIELDS):
    for k in fields:
        e = normwise(g, r, k)
        say(f"  {k}: max rel diff {e:.3e}")
        assert e <= tol, (k, e)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_absorbing_zones_on_every_wall_match_the_oracle(precision):
    c = I.case_c2(n=128, precision=precision)
    g, r = both(c, 60, (16.0, 10.0, 12.0, 20.0))
    if precision == "f64":
        # the FP64 kernels round as the oracle does: equal to the bit
        for k in FIELDS:
            assert np.array_equal(g[k], r[k]), k
    else:
        # the FP32 bar is on the depth and the discharges
        check(g, r, TOL32, ("h", "hu", "hv"))
        for k in ("w", "p"):
            say(f"  {k} (not held to the bar): {normwise(g, r, k):.3e}")


def test_channel_zone_absorbs_the_solitary_wave_as_the_oracle_does():
    c = I.case_c1()
    g, r = both(c, 660, (0.0, 6.0, 0.0, 0.0))
    check(g, r, TOL64, ("h", "hu", "w", "p"))
    x = (np.arange(c.nx) + 0.5) * c.dx
    eta = np.abs(g["h"][0] - c.H[0])[x < 10.0].max()
    assert eta < 0.01                  # the reflection is gone (0.1 without)


def test_given_targets_and_the_wall_cells_holding_them():
    c = I.case_c2(n=96)
    target = np.where(c.H > 0.0, c.H + 0.05, 0.0)   # raised; none on land
    g, r = both(c, 12, (8.0, 0.0, 0.0, 0.0), h=target)
    check(g, r, TOL64)
    assert np.array_equal(g["h"][:, 0], target[:, 0])


def test_zero_widths_switch_the_zones_off():
    from paper_1706_04551_amd import Solver
    c = I.case_c2(n=64)
    out = []
    for widths in (None, (0.0, 0.0, 0.0, 0.0), "on-then-off"):
        s = Solver.from_case(c)
        if widths == "on-then-off":
            s.set_relaxation((5.0, 5.0, 5.0, 5.0))
            s.set_relaxation((0.0, 0.0, 0.0, 0.0))
        elif widths is not None:
            s.set_relaxation(widths)
        s.run(8)
        out.append(s.state())
        s.close()
    for k in FIELDS:
        assert np.array_equal(out[0][k], out[1][k]), k
        assert np.array_equal(out[0][k], out[2][k]), k


def test_bad_widths_or_targets_are_rejected():
    from paper_1706_04551_amd import NhError, Solver
    c = I.case_c2(n=64)
    s = Solver.from_case(c)
    for widths in ((-1.0, 0, 0, 0), (float("nan"), 0, 0, 0),
                   (float("inf"), 0, 0, 0)):
        with pytest.raises(NhError):
            s.set_relaxation(widths)
    bad = c.H.copy()
    bad[3, 3] = float("nan")
    with pytest.raises(NhError):
        s.set_relaxation((4.0, 0, 0, 0), h=bad)
    s.set_relaxation((4.0, 0, 0, 0))   # still usable afterwards
    s.run(2)
    assert np.isfinite(s.state()["h"]).all()
    s.close()
