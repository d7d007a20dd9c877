"""Pins of the oracle's Manning friction against the exact solution of the
friction law.

On a flat bed with a uniform discharge and the pressure step off, the flux
terms cancel in every cell the walls have not yet reached (the stencil grows by
two cells per stage), so there the depth stays h0 and the discharge obeys the
friction law of Section 2 alone:
    q_t = -g n^2 |u| q / h0^(4/3),  |u| = |q| / h0,
whose exact solution keeps the direction of q and gives
    |q|(t) = |q0| / (1 + c |q0| t),  c = g n^2 / h0^(7/3).
The semi-implicit stages (averaged by the RK step) must converge to it.  A
dropped g or n^2, a wrong power of h, or a sign error converges to another
solution, or to none.
"""
import math

import numpy as np
import pytest

from oracle.oracle import Oracle, Params

G = 9.81
H0, Q0, N_MANNING, T_END = 0.5, 0.5, 0.1, 2.0


def interior_discharge(nx, ny, dx, dt, theta, manning=N_MANNING):
    steps = int(round(T_END / dt))
    reach = 4 * steps + 4  # cells the walls' influence can have crossed
    assert reach < nx // 2 and (ny == 1 or reach < ny // 2)
    P = Params(nx=nx, ny=ny, dx=dx, dy=dx, nh_on=0, fixed_dt=1, dt_fixed=dt,
               manning=manning)
    o = Oracle(P)
    shape = (ny, nx)
    o.set_bathymetry(np.full(shape, H0))
    hv = None if ny == 1 else np.full(shape, Q0 * math.sin(theta))
    o.set_state(np.full(shape, H0), np.full(shape, Q0 * math.cos(theta)), hv)
    assert o.run(steps) == 0
    s = o.state()
    j, i = ny // 2, nx // 2
    return s["h"][j, i], s["hu"][j, i], s["hv"][j, i]


def exact_speed(t):
    c = G * N_MANNING ** 2 / H0 ** (7.0 / 3.0)
    return Q0 / (1.0 + c * Q0 * t)


@pytest.mark.parametrize("ny,theta", [(1, 0.0), (160, math.pi / 6)])
def test_friction_converges_to_the_exact_decay(ny, theta):
    nx, dx = 160, 5.0
    errs = []
    for dt in (0.5, 0.25, 0.125):
        h, qa, qb = interior_discharge(nx, ny, dx, dt, theta)
        assert h == H0  # the flux terms cancel: depth unchanged
        speed = math.hypot(qa, qb)
        if ny > 1:  # the direction of q is kept
            assert math.atan2(qb, qa) == pytest.approx(theta, abs=1e-13)
        errs.append(abs(speed - exact_speed(T_END)))
    # first order in dt (semi-implicit stages: 1.1e-2, 5.6e-3, 2.8e-3)
    assert errs[2] < 1e-2 * Q0
    for a, b in zip(errs, errs[1:]):
        assert 1.9 < a / b < 2.1, errs


def test_zero_manning_leaves_the_discharge_unchanged():
    h, qa, qb = interior_discharge(160, 1, 5.0, 0.25, 0.0, manning=0.0)
    assert (h, qa) == (H0, Q0)


def test_negative_manning_is_rejected():
    with pytest.raises(ValueError):
        Oracle(Params(nx=8, ny=8, dx=1.0, dy=1.0, manning=-0.01))
