"""Pins of the oracle's generation/absorption zones (Section 4.4).

An absorbing zone must take out the waves that enter it: the solitary wave of
the 1D channel, reflected by the far wall without a zone, must come back
(nearly) without one.  A lake at rest with still-water targets stays at rest.
Widths of zero change nothing, and the cell at a wall, where the weight of the
state is zero, holds its target after every step.
"""
import numpy as np
import pytest

from oracle.oracle import Oracle, Params
from paper_1706_04551_amd import inputs as I


def oracle(case, widths=None, **targets):
    o = Oracle(Params(**case.param_dict()))
    o.set_bathymetry(case.H)
    o.set_state(case.h, case.hu, case.hv)
    if widths is not None:
        o.set_relaxation(widths, **targets)
    return o


def run_to(o, t_end):
    while o.stats()["t"] < t_end:
        assert o.step() == 0
    return o.state()


def test_absorbing_zone_takes_out_the_reflected_wave():
    # solitary wave of 0.1 m on 1 m, moving east in a 20 m channel; at
    # t = 9 s its reflection from the east wall is back in the west half
    c = I.case_c1()
    x = (np.arange(c.nx) + 0.5) * c.dx
    west = x < 10.0
    eta = {}
    for key, widths in (("wall", None), ("zone", (0.0, 6.0, 0.0, 0.0))):
        s = run_to(oracle(c, widths), 9.0)
        eta[key] = np.abs(s["h"][0] - c.H[0])[west].max()
    assert eta["wall"] > 0.08          # the reflected solitary wave
    assert eta["zone"] < 0.1 * eta["wall"], eta


def test_lake_at_rest_stays_at_rest_with_zones_on_every_wall():
    c = I.case_c2(n=96)
    c.h = np.maximum(c.H, 0.0)
    c.hu = np.zeros_like(c.H)
    c.hv = np.zeros_like(c.H)
    o = oracle(c, (12.0, 12.0, 12.0, 12.0))
    assert o.run(20) == 0
    s = o.state()
    assert np.abs(s["h"] - c.h).max() <= 1e-13
    assert np.abs(s["hu"]).max() <= 1e-13 and np.abs(s["hv"]).max() <= 1e-13


def test_zero_widths_change_nothing():
    c = I.case_c2(n=64)
    a = oracle(c)
    b = oracle(c, (0.0, 0.0, 0.0, 0.0))
    assert a.run(10) == 0 and b.run(10) == 0
    sa, sb = a.state(), b.state()
    for k in ("h", "hu", "hv", "w", "p"):
        assert np.array_equal(sa[k], sb[k]), k


def test_the_wall_cells_hold_their_target():
    c = I.case_c2(n=64)
    target = c.H + 0.05                 # a raised surface to relax towards
    o = oracle(c, (8.0, 0.0, 0.0, 0.0), h=target)
    for _ in range(5):
        assert o.step() == 0
        s = o.state()
        assert np.array_equal(s["h"][:, 0], target[:, 0])
        assert not np.array_equal(s["h"][:, 1], target[:, 1])


def test_negative_width_is_rejected():
    c = I.case_c2(n=64)
    with pytest.raises(ValueError):
        oracle(c, (-1.0, 0.0, 0.0, 0.0))
