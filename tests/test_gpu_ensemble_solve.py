"""The two forms of an ensemble's pressure solve on the GPU: one cooperative
launch per solve (solve_path 2: the sweep launches and the convergence
checks become phases of one kernel between grid barriers, no host decision
inside) and launches of 8 sweeps with the members still active read back at
every check (solve_path 1).  Both run the same blocks of sweeps and the same
checks, so every member's state, pressure, times, sweep counts and measure
agree to the bit; the members against their own single-grid solves too.
"""
import sys

import numpy as np
import pytest

from paper_1706_04551_amd import inputs as I

pytestmark = pytest.mark.gpu

FIELDS = ("h", "hu", "hv", "w", "p")
KEYS = ("t", "dt", "step", "sweeps1", "sweeps2", "sweeps_total", "solves",
        "measure", "status")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def members(precision, sides, **kw):
    out = []
    for k, n in enumerate(sides):
        c = I.case_c4_member(k, sides=(n,), precision=precision, island=True)
        for a, v in kw.items():
            setattr(c, a, v)
        out.append(c)
    return out


def both(cases, steps, label):
    from paper_1706_04551_amd import Ensemble
    say(f"[ensemble solve] {label}: {len(cases)} members, {steps} steps, "
        "solve_path 1 and 2")
    a = Ensemble.from_cases(cases, solve_path=1)
    b = Ensemble.from_cases(cases, solve_path=2)
    ra = a.run_status(steps)
    rb = b.run_status(steps)
    assert ra == rb, (ra, rb)
    for k in range(len(cases)):
        sa, sb = a.state(k), b.state(k)
        for f in FIELDS:
            assert np.array_equal(sa[f], sb[f]), (label, k, f)
        ta, tb = a.stats(k), b.stats(k)
        for key in KEYS:
            assert ta[key] == tb[key], (label, k, key, ta[key], tb[key])
    sw = [b.stats(k)["sweeps_total"] / max(1, b.stats(k)["solves"])
          for k in range(len(cases))]
    say("  equal to the bit; sweeps per solve " +
        " ".join(f"{x:.0f}" for x in sw))
    return a, b, ra


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_one_launch_equals_cycle_launches(precision):
    # uneven sides; the tolerances spread the members' stops over several
    # checks, so that members leave the solve at different phases
    cases = members(precision, (64, 97, 80, 130, 72))
    for k, c in enumerate(cases):
        c.solve_tol = (1e-8, 1e-10, 1e-9, 1e-11, 1e-7)[k] * (
            1e4 if precision == "f32" else 1.0)
    a, b, _ = both(cases, 12, f"mixed sides {precision}")
    a.close()
    b.close()


def test_one_launch_equals_single_grid_solves():
    from paper_1706_04551_amd import Ensemble, Solver
    cases = members("f64", (64, 97, 80))
    steps = 10
    e = Ensemble.from_cases(cases, solve_path=2)
    e.run(steps)
    for k, c in enumerate(cases):
        s = Solver.from_case(c)
        s.run(steps)
        for f in FIELDS:
            assert np.array_equal(e.state(k)[f], s.state()[f]), (k, f)
        assert e.stats(k)["sweeps_total"] == s.stats()["sweeps_total"]
        s.close()
    e.close()


def test_one_launch_with_periodic_and_breaking_members():
    cases = members("f64", (64, 80))
    cases[0].periodic = 3                # across the seam, island and all
    for c in cases:
        c.breaking_on = 1
    a, b, _ = both(cases, 8, "periodic + breaking")
    a.close()
    b.close()


def test_capped_solves_report_enoconv_in_both_forms():
    cases = members("f64", (64, 80))
    for c in cases:
        c.solve_max_iter = 40            # not a multiple of 8 or of 64
        c.solve_tol = 1e-30
    a, b, st = both(cases, 2, "capped at 40 sweeps")
    assert st == 0                       # the run goes on; the members say
    for k in range(len(cases)):
        assert b.stats(k)["status"] == -4
        assert b.stats(k)["sweeps1"] == 40 and b.stats(k)["sweeps2"] == 40
    a.close()
    b.close()


def test_check_every_sweep():
    cases = members("f64", (64, 72))
    for c in cases:
        c.omega = np.ones(1)             # plain Jacobi: checks every sweep
        c.check_every = 1
        c.solve_tol = 1e-9
    a, b, _ = both(cases, 4, "a check after every sweep")
    a.close()
    b.close()


def test_solve_path_is_shared_by_the_members():
    from paper_1706_04551_amd import Ensemble, NhError
    cases = members("f64", (64, 72))
    grids, params = [], []
    for j, c in enumerate(cases):
        kw = c.param_dict()
        grids.append((kw.pop("nx"), kw.pop("ny"), kw.pop("dx"), kw.pop("dy")))
        kw["precision"] = c.precision
        kw["solve_path"] = j + 1
        params.append(kw)
    with pytest.raises(NhError):
        Ensemble(grids, params)


def test_graph_replay_equals_run():
    # with one-launch solves a step waits for nothing on the host: captured
    # once into a graph and replayed, it gives nh_ensemble_run's results
    from paper_1706_04551_amd import Ensemble, NhError
    cases = members("f64", (64, 97, 80))
    cases[1].solve_tol = 1e-9
    say("[ensemble solve] graph replay of 3 members, 70 steps (a status "
        "read inside), solve_path 2")
    a = Ensemble.from_cases(cases, solve_path=2)
    b = Ensemble.from_cases(cases, solve_path=2)
    a.run(70)
    b.run_graph(30)
    b.run_graph(40)                       # the same graph, replayed again
    for k in range(len(cases)):
        for f in FIELDS:
            assert np.array_equal(a.state(k)[f], b.state(k)[f]), (k, f)
        for key in KEYS:
            assert a.stats(k)[key] == b.stats(k)[key], (k, key)
    # a new state rebuilds the tables, and the graph with them
    c = cases[0]
    a.set_state(0, c.h, c.hu, c.hv)
    b.set_state(0, c.h, c.hu, c.hv)
    a.run(5)
    b.run_graph(5)
    for f in FIELDS:
        assert np.array_equal(a.state(0)[f], b.state(0)[f]), f
    a.close()
    b.close()
    e = Ensemble.from_cases(cases[:1], solve_path=1)
    with pytest.raises(NhError):
        e.run_graph(1)
    e.close()


def test_a_wait_that_gives_up_ends_the_ensemble_run():
    # wait_polls < 0: every grid-barrier wait of the one-launch ensemble
    # solve gives up at once; the run reports NH_EDEVICE, eagerly and from
    # a graph replay, and a new ensemble runs
    from paper_1706_04551_amd import Ensemble, NhError
    cases = members("f64", (64, 72))
    say("[ensemble solve] forced give-up of the grid barriers")
    e = Ensemble.from_cases(cases, solve_path=2, wait_polls=-1)
    assert e.run_status(2) == -3
    e.close()
    e = Ensemble.from_cases(cases, solve_path=2, wait_polls=-1)
    with pytest.raises(NhError) as x:
        e.run_graph(2)
    assert x.value.status == -3
    e.close()
    ok = Ensemble.from_cases(cases, solve_path=2)
    assert ok.run_status(2) == 0
    ok.close()
