"""Pins of the oracle's energy-consistent vertical-momentum variant (the
form named after eq. 7: (hw)_t + div(hw u) = p, i.e. h (w_t + u . grad w) =
p), in the reading of the oracle: w is carried by the flow with first-order
upwinding at the corners in each stage's hyperbolic step.

The transport alone (hydrostatic mode, where w is passive): a uniform w stays
uniform under any flow; on a periodic channel with a uniform current the
total of w is conserved and its first moment moves by exactly u dt per step
(upwinding is exact for both; the Heun average adds a second difference,
whose first moment vanishes).  With the pressure step: a lake at rest is the
same in both forms to the bit, and a solitary wave (which moves) gives
another w than the model's form, and the same h to within the small
difference the transport of w makes.
"""
import math

import numpy as np
import pytest

from oracle.oracle import Oracle, Params
from paper_1706_04551_amd import inputs as I


def run(P, H, h, hu, hv, w, steps):
    o = Oracle(P)
    o.set_bathymetry(H)
    o.set_state(h, hu, hv, w)
    assert o.run(steps) == 0
    return o.state(), o.stats()


def test_uniform_w_stays_uniform_under_a_flow():
    rng = np.random.default_rng(7)
    nx, ny = 24, 20
    H, h, hu, hv = I.random_wet_state(rng, nx, ny, 1.0, 1.0)
    P = Params(nx=nx, ny=ny, dx=1.0, dy=1.0, nh_on=0, w_advection=1, cfl=0.5)
    w = np.full((ny + 1, nx + 1), 0.0375)
    s, _ = run(P, H, h, hu, hv, w, 30)
    assert np.all(s["w"] == 0.0375)


@pytest.mark.parametrize("u0", [0.4, -0.3])
def test_first_moment_moves_with_the_current(u0):
    # depth 2: the velocity is q / h, not q
    n, dx, steps = 200, 0.5, 40
    H = np.full((1, n), 2.0)
    P = Params(nx=n, ny=1, dx=dx, dy=1.0, nh_on=0, w_advection=1, periodic=1,
               fixed_dt=1, dt_fixed=0.05)
    xk = np.arange(n + 1) * dx
    w = np.exp(-((xk - 50.0) / 4.0) ** 2)
    w[n] = w[0]
    s, st = run(P, H, H.copy(), np.full((1, n), 2.0 * u0), None, w, steps)
    w1 = s["w"][:n]
    # upwinding is monotone: no new extrema
    assert w1.max() <= w.max() and w1.min() >= 0.0
    m0, m1 = w[:n].sum(), w1.sum()
    assert abs(m1 - m0) <= 1e-12 * m0
    shift = (xk[:n] * w1).sum() / m1 - (xk[:n] * w[:n]).sum() / m0
    assert abs(shift - u0 * st["t"]) <= 1e-9, (shift, u0 * st["t"])
    # and the model's form leaves w where it is (hydrostatic: no pressure)
    P0 = Params(nx=n, ny=1, dx=dx, dy=1.0, nh_on=0, periodic=1, fixed_dt=1,
                dt_fixed=0.05)
    s0, _ = run(P0, H, H.copy(), np.full((1, n), 2.0 * u0), None, w, steps)
    assert np.array_equal(s0["w"], w)


@pytest.mark.parametrize("u0,v0", [(0.3, -0.2), (-0.25, 0.35)])
def test_2d_transport_along_both_axes(u0, v0):
    # the bump stays far from the seams (first-order upwinding spreads it;
    # mass at a seam would enter the moment through the wrap-around)
    nx, ny, dx, dy = 56, 52, 1.0, 0.8
    H = np.ones((ny, nx))
    P = Params(nx=nx, ny=ny, dx=dx, dy=dy, nh_on=0, w_advection=1,
               periodic=3, fixed_dt=1, dt_fixed=0.1)
    X, Y = np.meshgrid(np.arange(nx + 1) * dx, np.arange(ny + 1) * dy)
    w = np.exp(-((X - 28.0) ** 2 + (Y - 20.8) ** 2) / 9.0)
    w[:, nx] = w[:, 0]
    w[ny, :] = w[0, :]
    s, st = run(P, H, H.copy(), np.full((ny, nx), u0), np.full((ny, nx), v0),
                w, 30)
    a, b = w[:ny, :nx], s["w"][:ny, :nx]
    assert abs(b.sum() - a.sum()) <= 1e-12 * a.sum()
    for coord, vel in ((X[:ny, :nx], u0), (Y[:ny, :nx], v0)):
        shift = (coord * b).sum() / b.sum() - (coord * a).sum() / a.sum()
        assert abs(shift - vel * st["t"]) <= 1e-9, (shift, vel * st["t"])


def test_lake_at_rest_is_the_same_in_both_forms():
    c = I.case_c2(n=160)            # with the dry island
    c.h = np.maximum(c.H, 0.0)
    out = []
    for wa in (0, 1):
        kw = c.param_dict()
        kw["w_advection"] = wa
        s, _ = run(Params(**kw), c.H, c.h, c.hu, c.hv, None, 20)
        out.append(s)
    for k in ("h", "hu", "hv", "w", "p"):
        assert np.array_equal(out[0][k], out[1][k]), k


def test_moving_wave_changes_w_but_barely_h():
    c = I.case_c1(steps=200)
    res = []
    for wa in (0, 1):
        kw = c.param_dict()
        kw["w_advection"] = wa
        s, _ = run(Params(**kw), c.H, c.h, c.hu, c.hv, None, c.steps)
        res.append(s)
    dw = np.abs(res[1]["w"] - res[0]["w"]).max() / np.abs(res[0]["w"]).max()
    dh = np.abs(res[1]["h"] - res[0]["h"]).max() / 0.1   # of the amplitude
    assert dw > 1e-3, dw          # the transport of w is there
    assert dh < 1e-2, dh          # and the wave is the same wave


def test_invalid_flag_is_refused():
    with pytest.raises(Exception):
        Oracle(Params(nx=8, ny=6, dx=1.0, dy=1.0, w_advection=2))


@pytest.mark.parametrize("wadv", [0, 1])
def test_discrete_energy_never_grows_on_a_flat_bed(wadv):
    # the energy of the depth-averaged system with its vertical momentum,
    # sum (g h^2 / 2 + |q|^2 / (2 h) + h w^2 / 2) dx dy (w at the cell as the
    # mean of its corners), of a Gaussian hump in a closed flat basin: the
    # scheme only dissipates it (upwinded fluxes, the projection), in both
    # forms of the w equation, step by step, by more than rounding
    n, g = 48, 9.81
    c = I.case_c2(n=n, island=False)
    c.H = np.ones_like(c.H)
    xc = (np.arange(n) + 0.5) * c.dx
    X, Y = np.meshgrid(xc, xc)
    L = n * c.dx
    c.h = c.H + 0.2 * np.exp(-((X - L / 2) ** 2 + (Y - L / 2) ** 2)
                             / (0.1 * L) ** 2)
    c.w_advection = wadv
    c.solve_tol = 1e-13
    o = Oracle(Params(**c.param_dict()))
    o.set_bathymetry(c.H)
    o.set_state(c.h, c.hu, c.hv)

    def energy():
        s = o.state()
        h, hu, hv, w = s["h"], s["hu"], s["hv"], s["w"]
        wc = 0.25 * (w[:-1, :-1] + w[1:, :-1] + w[:-1, 1:] + w[1:, 1:])
        return float(np.sum(0.5 * g * h * h + 0.5 * (hu * hu + hv * hv) / h
                            + 0.5 * h * wc * wc)) * c.dx * c.dy

    E = [energy()]
    for _ in range(120):
        assert o.step() == 0
        E.append(energy())
    d = np.diff(np.array(E))
    assert d.max() <= 1e-12 * E[0], d.max()
    assert E[-1] < E[0]   # and some of it is dissipated
