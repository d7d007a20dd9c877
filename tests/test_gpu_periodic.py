"""Periodic boundaries (Section 4.4, item 1) on the GPU against the FP64
oracle, whose periodic boundaries are pinned (cyclic shifts commute with a
run, a uniform current stays uniform, mass is conserved, the cyclic 1D solve
equals a dense one, the linear dispersion relation holds on a periodic
channel).  FP64 is compared to the bit, FP32 to 1e-4 on h and the
discharges; single grids and ensemble members; ragged sweep tiles whose
halos wrap around.
"""
import sys

import numpy as np
import pytest

from oracle.oracle import Oracle, Params
from paper_1706_04551_amd import inputs as I

pytestmark = pytest.mark.gpu

FIELDS = ("h", "hu", "hv", "w", "p")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def normwise(g, r, k):
    scale = np.abs(r[k]).max()
    if k in ("hu", "hv"):
        scale = max(np.abs(r["hu"]).max(), np.abs(r["hv"]).max())
    return float(np.abs(g[k] - r[k]).max() / max(scale, 1e-300))


def gpu_state(case, steps):
    from paper_1706_04551_amd import Solver
    s = Solver.from_case(case)
    s.run(steps)
    out, st = s.state(), s.stats()
    s.close()
    return out, st


def oracle_state(case, steps):
    o = Oracle(Params(**case.param_dict()))
    o.set_bathymetry(case.H)
    o.set_state(case.h, case.hu, case.hv)
    assert o.run(steps) == 0
    return o.state(), o.stats()


def basin(n, periodic, precision="f64"):
    c = I.case_c2(n=n, precision=precision, island=False)
    c.periodic = periodic
    return c


@pytest.mark.parametrize("n,periodic", [(96, 1), (97, 3), (130, 2)])
def test_periodic_basin_equals_the_oracle_fp64(n, periodic):
    # 97 and 130 corners per side: ragged sweep tiles whose halos wrap
    c = basin(n, periodic)
    steps = 25
    say(f"[case] basin {n}x{n} periodic={periodic} f64, {steps} steps")
    g, gs = gpu_state(c, steps)
    r, rs = oracle_state(c, steps)
    for k in FIELDS:
        assert np.array_equal(g[k], r[k]), (k, normwise(g, r, k))
    assert gs["t"] == rs["t"] and gs["sweeps_total"] == rs["sweeps_total"]
    if periodic & 1:
        assert np.array_equal(g["p"][:, 0], g["p"][:, n])
    if periodic & 2:
        assert np.array_equal(g["w"][0, :], g["w"][n, :])


def test_periodic_basin_fp32():
    c = basin(96, 3, "f32")
    steps = 25
    say(f"[case] basin 96x96 periodic=3 f32, {steps} steps")
    g, _ = gpu_state(c, steps)
    r, _ = oracle_state(c, steps)
    for k in ("h", "hu", "hv"):
        e = normwise(g, r, k)
        say(f"  {k}: {e:.2e}")
        assert e <= 1e-4, (k, e)


def test_periodic_channel_equals_the_oracle():
    # the 1D channel with its cyclic pressure system: the solitary wave
    # crosses the seam
    c = I.case_c1(steps=600)
    c.periodic = 1
    say("[case] channel 400 cells periodic, 600 steps")
    g, _ = gpu_state(c, c.steps)
    r, _ = oracle_state(c, c.steps)
    for k in ("h", "hu", "w", "p"):
        e = normwise(g, r, k)
        say(f"  {k}: {e:.2e}")
        assert np.array_equal(g[k], r[k].reshape(g[k].shape)), (k, e)
    assert g["p"][0] == g["p"][-1]


def test_gpu_run_commutes_with_cyclic_shifts():
    # the property the oracle is pinned by, on the GPU: to the bit in 2D
    c = basin(80, 3)
    steps, sx, sy = 20, 29, 11
    a, _ = gpu_state(c, steps)
    sh = lambda x: np.roll(np.roll(x, sx, axis=1), sy, axis=0)  # noqa: E731
    c2 = basin(80, 3)
    c2.H, c2.h, c2.hu, c2.hv = sh(c.H), sh(c.h), sh(c.hu), sh(c.hv)
    b, _ = gpu_state(c2, steps)
    for k in ("h", "hu", "hv"):
        assert np.array_equal(sh(a[k]), b[k]), k
    for k in ("w", "p"):
        assert np.array_equal(sh(a[k][:80, :80]), b[k][:80, :80]), k


def test_ensemble_members_with_periodic_directions():
    from paper_1706_04551_amd import Ensemble
    cases = [basin(n, per) for n, per in ((64, 1), (72, 3), (80, 0))]
    steps = 10
    e = Ensemble.from_cases(cases)
    e.run(steps)
    for k, c in enumerate(cases):
        r, _ = gpu_state(c, steps)
        g = e.state(k)
        for f in FIELDS:
            assert np.array_equal(g[f], r[f]), (k, f)
    e.close()


def test_invalid_periodic_settings_are_refused():
    from paper_1706_04551_amd import NhError, Solver
    with pytest.raises(NhError):
        Solver(16, 16, 1.0, 1.0, periodic=4)
    with pytest.raises(NhError):
        Solver(16, 16, 1.0, 1.0, periodic=1, open_sides=2)
    s = Solver(16, 16, 1.0, 1.0, periodic=1)
    s.set_bathymetry(np.ones((16, 16)))
    with pytest.raises(NhError):
        s.set_relaxation((2.0, 0.0, 0.0, 0.0))
    s.close()
