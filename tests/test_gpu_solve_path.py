"""The two launch forms of the 2D pressure solve on the GPU: one cooperative
launch per solve (solve_path 2: each workgroup keeps its tile's rows on chip,
convergence decided on the device) and launches of 8 sweeps with the
measure read back at each check (solve_path 1).  Both run the relaxation of
eq. (32) with the same schedule and checks, so states, pressures, times and
sweep counts agree to the bit; against the FP64 oracle the one-launch form
is compared to the bit as well.  Cases: walls with a dry island, open
sides, periodic lines (the last corner is the first one again), ragged
tiles, FP32 bulk, breaking, a capped solve, two solvers on one stream.
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


def solver(case, path, **over):
    from paper_1706_04551_amd import Solver
    return Solver.from_case(case, solve_path=path, **over)


def oracle_for(case):
    o = Oracle(Params(**case.param_dict()))
    o.set_bathymetry(case.H)
    o.set_state(case.h, case.hu, case.hv)
    return o


def same_runs(case, steps, label):
    say(f"[case] {label}: {steps} steps, solve_path 1 and 2")
    a = solver(case, 1)
    b = solver(case, 2)
    a.run(steps)
    b.run(steps)
    sa, sb = a.state(), b.state()
    ta, tb = a.stats(), b.stats()
    for k in FIELDS:
        assert np.array_equal(sa[k], sb[k]), (label, k,
                                              np.abs(sa[k] - sb[k]).max())
    for k in ("t", "step", "sweeps1", "sweeps2", "sweeps_total", "solves",
              "measure"):
        assert ta[k] == tb[k], (label, k, ta[k], tb[k])
    say(f"  equal to the bit; mean sweeps per solve "
        f"{ta['sweeps_total'] / max(ta['solves'], 1):.1f}")
    return sa, ta


def basin(n, precision="f64", island=True, **kw):
    c = I.case_c2(n=n, precision=precision, island=island)
    for k, v in kw.items():
        setattr(c, k, v)
    return c


@pytest.mark.parametrize("n,island,kw", [
    (96, True, {}),
    (130, True, {}),                   # ragged tiles
    (61, False, {"open_sides": 15}),
    (96, False, {"periodic": 1}),
    (97, False, {"periodic": 3}),
    (70, False, {"periodic": 2, "open_sides": 3}),
])
def test_one_launch_equals_cycle_launches_fp64(n, island, kw):
    c = basin(n, island=island, **kw)
    same_runs(c, 40, f"basin {n} island={island} {kw} f64")


def test_plain_and_cooperative_one_launch_agree():
    # solve_path 0 launches the one-launch solve plainly (no more
    # workgroups than are co-resident), 2 cooperatively: the same kernel
    c = basin(130)
    say("[case] basin 130: solve_path 0 (plain launch) and 2 (cooperative)")
    a = solver(c, 0)
    b = solver(c, 2)
    a.run(30)
    b.run(30)
    for k in FIELDS:
        assert np.array_equal(a.state()[k], b.state()[k]), k
    for k in ("t", "sweeps_total", "measure"):
        assert a.stats()[k] == b.stats()[k], k


def test_one_launch_equals_cycle_launches_fp32():
    c = basin(96, precision="f32")
    same_runs(c, 40, "basin 96 f32")


def test_one_launch_with_breaking_and_small_checks():
    c = basin(64, island=False)
    c.breaking_on = 1
    c.omega = np.ones(1)
    c.check_every = 1                 # a grid-wide decision every sweep
    c.solve_tol = 1e-9
    same_runs(c, 10, "basin 64 breaking, check every sweep")


def test_one_launch_equals_the_oracle_fp64():
    c = basin(96)
    steps = 30
    say(f"[case] basin 96 island f64 vs oracle, {steps} steps (solve_path 2)")
    g = solver(c, 2)
    o = oracle_for(c)
    g.run(steps)
    assert o.run(steps) == 0
    sg, so = g.state(), o.state()
    for k in FIELDS:
        assert np.array_equal(sg[k], so[k]), (k, np.abs(sg[k] - so[k]).max())
    assert g.stats()["t"] == o.stats()["t"]
    assert g.stats()["sweeps_total"] == o.stats()["sweeps_total"]


def test_one_launch_periodic_equals_the_oracle():
    c = basin(97, island=False, periodic=3)
    steps = 20
    say(f"[case] basin 97 periodic 3 vs oracle, {steps} steps (solve_path 2)")
    g = solver(c, 2)
    o = oracle_for(c)
    g.run(steps)
    assert o.run(steps) == 0
    sg, so = g.state(), o.state()
    for k in FIELDS:
        assert np.array_equal(sg[k], so[k]), (k, np.abs(sg[k] - so[k]).max())
    # the last corner of each periodic line is its first one again
    assert np.array_equal(sg["p"][:, -1], sg["p"][:, 0])
    assert np.array_equal(sg["p"][-1, :], sg["p"][0, :])


def test_capped_solve_reports_enoconv_and_keeps_the_state():
    c = basin(64)
    c.solve_max_iter = 64
    c.solve_tol = 1e-30
    say("[case] capped solves: status NH_ENOCONV from both launch forms")
    a = solver(c, 1)
    b = solver(c, 2)
    assert a.run_status(1) == -4
    assert b.run_status(1) == -4
    sa, sb = a.state(), b.state()
    for k in FIELDS:
        assert np.array_equal(sa[k], sb[k]), k
    assert b.stats()["sweeps1"] == 64 and b.stats()["sweeps2"] == 64
    # the state stays valid: the next steps run and are capped again.  The
    # cycle launches stop at the first capped step; the one launch per
    # solve reports it at the next status read, here the end of the run
    assert b.run_status(2) == -4
    assert b.stats()["step"] == 3
    assert a.run_status(1) == -4 and a.run_status(1) == -4
    assert a.stats()["step"] == 3
    assert np.array_equal(a.state()["h"], b.state()["h"])
    o = oracle_for(c)
    assert o.step() == -4
    assert np.array_equal(sa["h"], o.state()["h"])


def test_two_solvers_alternate_on_one_stream():
    c1 = basin(80)
    c2 = basin(48, island=False, periodic=1)
    say("[case] two one-launch solvers alternating on torch's stream")
    import torch
    st = torch.cuda.current_stream().cuda_stream
    from paper_1706_04551_amd import Solver
    a = Solver.from_case(c1, solve_path=2, stream=st)
    b = Solver.from_case(c2, solve_path=2, stream=st)
    for _ in range(5):
        a.run(3)
        b.run(3)
    ra = solver(c1, 1)
    rb = solver(c2, 1)
    ra.run(15)
    rb.run(15)
    for k in FIELDS:
        assert np.array_equal(a.state()[k], ra.state()[k]), k
        assert np.array_equal(b.state()[k], rb.state()[k]), k


def test_set_state_restarts_the_one_launch_solve():
    c = basin(64)
    say("[case] set_state between runs of a one-launch solver")
    a = solver(c, 2)
    a.run(5)
    a.set_state(c.h, c.hu, c.hv)
    a.run(5)
    b = solver(c, 1)
    b.run(5)
    for k in FIELDS:
        assert np.array_equal(a.state()[k], b.state()[k]), k
    assert a.stats()["step"] == 5


def test_solve_path_checks():
    from paper_1706_04551_amd import NhError, Solver
    with pytest.raises(NhError) as e:
        Solver(16, 16, 1.0, 1.0, solve_path=3)
    assert e.value.status == -1
    # 1024^2 cells: more tiles than co-resident workgroups
    with pytest.raises(NhError) as e:
        Solver(1024, 1024, 1.0, 1.0, solve_path=2)
    assert e.value.status == -1
    # the automatic choice takes the cycle launches there
    s = Solver(1024, 1024, 1.0, 1.0, solve_path=0)
    s.close()


@pytest.mark.parametrize("path", [1, 2])
def test_relative_residual_stop_equals_the_oracle(path):
    # solve_norm 1: the solves stop on max |rhs - A p| / max |rhs|; the GPU
    # (either launch form) takes the oracle's decisions and so its iterates,
    # sweep counts and state to the bit
    c = basin(96)
    c.solve_norm = 1
    c.solve_tol = 1e-9
    steps = 15
    say(f"[case] basin 96, relative-residual stop, solve_path {path}")
    g = solver(c, path)
    o = oracle_for(c)
    g.run(steps)
    assert o.run(steps) == 0
    sg, so = g.state(), o.state()
    for k in FIELDS:
        assert np.array_equal(sg[k], so[k]), (k, np.abs(sg[k] - so[k]).max())
    gs, os_ = g.stats(), o.stats()
    assert gs["sweeps_total"] == os_["sweeps_total"]
    assert gs["measure"] == os_["measure"] and gs["measure"] < 1e-9
    # and another measure than the default one (with checks every 64
    # sweeps both may stop at the same check)
    c0 = basin(96)
    c0.solve_tol = 1e-9
    g0 = solver(c0, path)
    g0.run(steps)
    assert g0.stats()["measure"] != gs["measure"]


def test_relative_residual_stop_is_refused_where_not_built():
    from paper_1706_04551_amd import Ensemble, NhError, Solver
    with pytest.raises(NhError):
        Solver(16, 16, 1.0, 1.0, solve_norm=2)
    c = basin(64)
    c.solve_norm = 1
    with pytest.raises(NhError):
        Ensemble.from_cases([c, c])
    s = solver(c, 0)
    with pytest.raises(NhError):
        s.adjoint(2, [5], np.zeros((2, 1)), ckpt_every=1)


@pytest.mark.parametrize("path", [0, 2])
def test_a_wait_that_gives_up_ends_the_run(path):
    # wait_polls < 0 makes every wait between workgroups give up at once:
    # every workgroup leaves the launch, the run reports NH_EDEVICE at its
    # next status read and the solver refuses further steps; the device
    # stays usable
    c = basin(64)
    say(f"[case] forced give-up of the one-launch solve, solve_path {path}")
    s = solver(c, path, wait_polls=-1)
    assert s.run_status(3) == -3
    assert s.run_status(1) == -8
    s.close()
    ok = solver(c, path)
    assert ok.run_status(3) == 0
    ok.close()
