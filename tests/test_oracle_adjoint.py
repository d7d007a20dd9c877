"""Pins of the differentiable oracle (oracle/nh_torch.py), CPU only.

The torch statement of the 2D step uses the literal corner constraint (eq. 37
with eq. 36 and 41 substituted) and a dense solve; the C oracle uses the
closed-form five-point rows and relaxed Jacobi.  They must give the same
states.  Its reverse-mode gradient of a gauge misfit must match central
differences of the C oracle (the derivative the paper's scheme defines away
from limiter kinks) and its forward-mode tangent (dot-product test).
"""
import numpy as np
import pytest

from oracle import nh_torch as NT
from oracle.oracle import Oracle, Params
from paper_1706_04551_amd import inputs as I


def c_oracle(nx, ny, dx, dy, dt, **kw):
    par = dict(nx=nx, ny=ny, dx=dx, dy=dy, cfl=0.7, solve_tol=1e-14,
               solve_max_iter=400000, check_every=1, fixed_dt=1, dt_fixed=dt)
    par.update(kw)
    return Oracle(Params(**par))


def test_torch_step_equals_c_oracle_on_a_wet_state():
    rng = np.random.default_rng(3)
    nx, ny, dx, dy, dt, steps = 13, 11, 1.0, 1.2, 0.02, 5
    H, h, hu, hv = I.random_wet_state(rng, nx, ny, dx, dy)
    o = c_oracle(nx, ny, dx, dy, dt)
    o.set_bathymetry(H)
    o.set_state(h, hu, hv)
    assert o.run(steps) == 0
    r = o.state()
    s = NT.run(NT.TorchParams(nx, ny, dx, dy, dt), h, hu, hv, H, steps)
    for k in ("h", "hu", "hv", "w"):
        assert np.abs(s[k] - r[k]).max() <= 1e-13 * np.abs(r[k]).max(), k
    assert np.abs(s["p"] - r["p"]).max() <= 1e-11 * np.abs(r["p"]).max()


def test_torch_step_equals_c_oracle_with_dry_land():
    # the island basin at a small size: dry cells, emerging bed, wet-dry
    # slopes and a hump of 0.5 m; the fixed dt is below the CFL limit
    H, h = I.island_basin(64, 1.0, 7, hump_amp=0.5)
    z = np.zeros_like(h)
    dt, steps = 0.02, 4
    o = c_oracle(64, 64, 1.0, 1.0, dt, solve_tol=1e-13)
    o.set_bathymetry(H)
    o.set_state(h, z, z)
    assert o.run(steps) == 0
    assert (h == 0).any()
    r = o.state()
    s = NT.run(NT.TorchParams(64, 64, 1.0, 1.0, dt), h, z, z, H, steps)
    for k in ("h", "hu", "hv"):
        scale = np.abs(r[k]).max()
        assert np.abs(s[k] - r[k]).max() <= 1e-10 * scale, k


def misfit_problem():
    rng = np.random.default_rng(4)
    nx, ny, dx, dy = 12, 10, 2.0, 2.0
    H, _, _, _ = I.random_wet_state(rng, nx, ny, dx, dy, depth=(3.0, 8.0))
    x = (np.arange(nx) + 0.5)[None, :]
    y = (np.arange(ny) + 0.5)[:, None]
    # bump centre off the cell lattice: no limiter tie at the base point
    eta0 = 0.3 * np.exp(-((x - 6.37) ** 2 + (y - 4.71) ** 2) / 8.0)
    dt, steps = 0.05, 8
    gauges = np.array([3 * nx + 4, 6 * nx + 8, 2 * nx + 10])
    target = (0.01 * rng.standard_normal((steps, 3)) +
              (H + eta0).reshape(-1)[gauges][None, :])
    return nx, ny, dx, dy, dt, steps, H, eta0, gauges, target


def c_misfit(nx, ny, dx, dy, dt, steps, H, eta0, gauges, target):
    o = c_oracle(nx, ny, dx, dy, dt)
    o.set_bathymetry(H)
    z = np.zeros_like(H)
    o.set_state(np.maximum(H + eta0, 0.0), z, z)
    J = 0.0
    for n in range(steps):
        assert o.step() == 0
        r = o.state()["h"].reshape(-1)[gauges] - target[n]
        J += 0.5 * float(np.sum(r * r))
    return J


def test_misfit_equals_c_oracle():
    nx, ny, dx, dy, dt, steps, H, eta0, gauges, target = misfit_problem()
    P = NT.TorchParams(nx, ny, dx, dy, dt)
    Jt = float(NT.misfit(P, NT.torch.as_tensor(eta0), NT.torch.as_tensor(H),
                         gauges, target, steps))
    Jc = c_misfit(nx, ny, dx, dy, dt, steps, H, eta0, gauges, target)
    assert abs(Jt - Jc) <= 1e-12 * Jc


@pytest.mark.parametrize("which", ["eta0", "H", "both"])
def test_gradient_matches_central_differences_of_the_c_oracle(which):
    nx, ny, dx, dy, dt, steps, H, eta0, gauges, target = misfit_problem()
    P = NT.TorchParams(nx, ny, dx, dy, dt)
    J, ge, gb = NT.gradient(P, eta0, H, gauges, target, steps)
    rng = np.random.default_rng({"eta0": 11, "H": 12, "both": 13}[which])
    de = rng.standard_normal(eta0.shape) if which != "H" else np.zeros_like(H)
    db = rng.standard_normal(H.shape) if which != "eta0" else np.zeros_like(H)
    eps = 1e-7
    fd = (c_misfit(nx, ny, dx, dy, dt, steps, H + eps * db, eta0 + eps * de,
                   gauges, target) -
          c_misfit(nx, ny, dx, dy, dt, steps, H - eps * db, eta0 - eps * de,
                   gauges, target)) / (2 * eps)
    ad = float(np.sum(ge * de) + np.sum(gb * db))
    assert abs(fd - ad) <= 1e-5 * abs(ad), (fd, ad)


def test_tangent_linear_model_equals_the_adjoint():
    nx, ny, dx, dy, dt, steps, H, eta0, gauges, target = misfit_problem()
    P = NT.TorchParams(nx, ny, dx, dy, dt)
    _, ge, gb = NT.gradient(P, eta0, H, gauges, target, steps)
    rng = np.random.default_rng(21)
    de = rng.standard_normal(eta0.shape)
    db = rng.standard_normal(H.shape)
    _, tl = NT.tangent(P, eta0, H, de, db, gauges, target, steps)
    ad = float(np.sum(ge * de) + np.sum(gb * db))
    assert abs(tl - ad) <= 1e-12 * abs(ad)


def test_torch_friction_equals_the_c_oracle():
    """The differentiable oracle's friction against the C oracle's (pinned
    to the exact decay of the friction law), on the island basin."""
    from oracle.oracle import Oracle, Params
    from paper_1706_04551_amd import inputs as I
    c = I.case_c2(n=64)
    dt = 0.02
    P = NT.TorchParams(c.nx, c.ny, c.dx, c.dy, dt, manning=0.05)
    s = NT.run(P, c.h, c.hu, c.hv, c.H, 6)
    o = Oracle(Params(**{**c.param_dict(), "fixed_dt": 1, "dt_fixed": dt,
                         "manning": 0.05, "solve_tol": 1e-13}))
    o.set_bathymetry(c.H)
    o.set_state(c.h, c.hu, c.hv)
    assert o.run(6) == 0
    r = o.state()
    for k in ("h", "hu", "hv"):
        assert np.abs(s[k] - r[k]).max() <= 1e-12 * np.abs(r[k]).max(), k
