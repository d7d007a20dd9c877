"""Seeded synthetic inputs: bathymetry, initial states and solver parameters.

This module is shared by the GPU path and the CPU oracle and holds none of the
scheme's arithmetic: it only draws and shapes input arrays (numpy PCG64
generators with fixed seeds) and builds parameter arrays (the relaxation
schedule) that the caller hands to either side.  Both sides therefore consume
exactly the same arrays.

Workloads (the paper's lab data are not available; these synthetic stand-ins
have the shapes of its workloads):
  c1  1D channel, solitary wave of eq. (33) (Section 7.1 shape), walls.
  c2  2D 512x512, smooth random bathymetry with a dry island and a Gaussian
      hump (circular dam-break / conical-island shapes of Sections 7.6-7.7).
  c3  2D 2048x2048 plane beach with an incoming solitary wave, breaking on
      (Section 7.4 shape).
  c4  ensemble of 64 c2-like basins of uneven sides 128-1024, FP32 bulk.
  c5  1024x1024 fully wet basin (dx 10 m, depth 5-50 m), fixed dt, gauges:
      the adjoint workload.
Cell centres sit at ((i+1/2) dx, (j+1/2) dy).  Arrays are [ny][nx], float64.

CFL: the 1D channel uses 0.9.  The 2D workloads use 0.7: with the 2D time
step taken from the sum of the x and y wave-speed ratios, the second-order
Runge-Kutta stage with dimension-wise MUSCL reconstruction lets round-off
perturbations grow (about x1.8 per step on these grids) for CFL above ~0.75.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

G = 9.81
CFL_2D = 0.7
SEED_C2 = 170604551
SEED_C4 = 170604552
SEED_C5 = 170604553


@dataclass
class Case:
    """A workload: grid, bathymetry, initial state and scheme parameters."""
    name: str
    nx: int
    ny: int
    dx: float
    dy: float
    H: np.ndarray
    h: np.ndarray
    hu: np.ndarray
    hv: np.ndarray
    steps: int
    g: float = G
    cfl: float = 0.9
    delta: float = 1e-5
    dry_eps: float = 1e-10
    nh_on: int = 1
    breaking_on: int = 0
    b1: float = 0.15
    b2: float = 0.5
    solve_tol: float = 1e-10
    solve_max_iter: int = 200000
    check_every: int = 1
    omega: np.ndarray = field(default_factory=lambda: np.ones(1))
    precision: str = "f64"
    fixed_dt: int = 0
    dt_fixed: float = 0.0
    manning: float = 0.0    # Gauckler-Manning n (0: no friction)
    open_sides: int = 0     # outflow sides: 1 west, 2 east, 4 south, 8 north
    periodic: int = 0       # periodic directions: 1 x, 2 y
    w_advection: int = 0    # 1: (hw)_t + div(hw u) = p instead of h w_t = p
    solve_norm: int = 0     # 1: stop on the relative residual, not eq. (32)

    def param_dict(self) -> dict:
        return dict(nx=self.nx, ny=self.ny, dx=self.dx, dy=self.dy, g=self.g,
                    cfl=self.cfl, delta=self.delta, dry_eps=self.dry_eps,
                    nh_on=self.nh_on, breaking_on=self.breaking_on,
                    b1=self.b1, b2=self.b2, solve_max_iter=self.solve_max_iter,
                    check_every=self.check_every, solve_tol=self.solve_tol,
                    omega=self.omega, fixed_dt=self.fixed_dt,
                    dt_fixed=self.dt_fixed, manning=self.manning,
                    open_sides=self.open_sides, periodic=self.periodic,
                    w_advection=self.w_advection, solve_norm=self.solve_norm)


# --------------------------------------------------------------------------
# relaxation schedule (a solver parameter, handed to both sides)
# --------------------------------------------------------------------------
def leja_order(x: np.ndarray) -> np.ndarray:
    """Leja ordering of points (start with the largest magnitude, then
    greedily maximise the product of distances to the points already taken).
    Used to order the factors of a Richardson/Jacobi polynomial so that the
    intermediate growth of the error stays bounded."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    left = list(range(n))
    first = int(np.argmax(np.abs(x)))
    order = [first]
    left.remove(first)
    logd = np.zeros(n)
    while left:
        for i in left:
            logd[i] += math.log(abs(x[i] - x[order[-1]]) + 1e-300)
        nxt = max(left, key=lambda i: logd[i])
        order.append(nxt)
        left.remove(nxt)
    return x[np.array(order)]


def srj_schedule(rho: float, m: int) -> np.ndarray:
    """Relaxation factors for m Jacobi sweeps: the reciprocals of the roots of
    the degree-m Chebyshev polynomial on [1 - rho, 1 + rho] (the interval that
    holds the spectrum of D^-1 A when the Jacobi iteration matrix has spectral
    radius rho), in Leja order.  A cycle of m sweeps then applies the scaled
    Chebyshev polynomial to the error."""
    if m == 1:
        return np.ones(1)
    k = np.arange(1, m + 1)
    lam = 1.0 + rho * np.cos((2 * k - 1) * math.pi / (2 * m))
    return 1.0 / leja_order(lam)


def jacobi_radius_bound(h_max: float, dx: float, dy: float | None,
                        margin: float = 1.0) -> float:
    """Estimate of the Jacobi iteration radius of the pressure system from
    the largest depth: off-diagonal over diagonal weight of a flat row,
    8 h^2 (1/dx^2 + 1/dy^2) / (16 + 8 h^2 (1/dx^2 + 1/dy^2)), with the depth
    scaled by `margin`.  On the 512^2 basin a margin of 1.1 costs 17 % more
    sweeps per solve than 1.0 at the same tolerance; both converge."""
    hh = (h_max * margin) ** 2
    s = hh / dx ** 2 if dy is None else hh * (1.0 / dx ** 2 + 1.0 / dy ** 2)
    return 8.0 * s / (16.0 + 8.0 * s)


# --------------------------------------------------------------------------
# building blocks
# --------------------------------------------------------------------------
def centres(n: int, d: float) -> np.ndarray:
    return (np.arange(n) + 0.5) * d


def solitary_wave(x: np.ndarray, A: float, H: float, x0: float, g: float = G):
    """Initial surface and velocity of eq. (33) at t = 0 (an approximate
    solitary wave, used only as initial data)."""
    eta = A / np.cosh(math.sqrt(3.0 * A / (4.0 * H ** 3)) * (x - x0)) ** 2
    u = math.sqrt(g * H) / H * eta
    return eta, u


def gaussian_field(rng: np.random.Generator, nx: int, ny: int, L_x: float,
                   L_y: float, xc: np.ndarray, yc: np.ndarray,
                   n_bumps: int = 8) -> np.ndarray:
    """Normalised sum of n_bumps random Gaussians on the domain, in [0, 1].
    Amplitudes U[0.5, 1], widths U[30, 90]/512 of the domain side, centres
    uniform over the domain."""
    L = max(L_x, L_y)
    a = rng.uniform(0.5, 1.0, n_bumps)
    s = rng.uniform(30.0, 90.0, n_bumps) * (L / 512.0)
    cx = rng.uniform(0.0, L_x, n_bumps)
    cy = rng.uniform(0.0, L_y, n_bumps)
    X, Y = np.meshgrid(xc, yc)
    D = np.zeros((ny, nx))
    for k in range(n_bumps):
        D += a[k] * np.exp(-((X - cx[k]) ** 2 + (Y - cy[k]) ** 2) /
                           (2.0 * s[k] ** 2))
    return (D - D.min()) / (D.max() - D.min())


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
def case_c1(steps: int = 300) -> Case:
    """1D channel: 400 cells, dx = 0.05 m, flat depth 1 m, solitary wave of
    amplitude 0.1 m centred at x = 5 m with the velocity of eq. (33), w = p = 0,
    CFL 0.9, walls."""
    nx, dx = 400, 0.05
    x = centres(nx, dx)
    eta, u = solitary_wave(x, 0.1, 1.0, 5.0)
    H = np.ones((1, nx))
    h = (1.0 + eta)[None, :]
    hu = h * u[None, :]
    return Case("c1", nx, 1, dx, 1.0, H, h, hu, np.zeros_like(h), steps,
                solve_tol=1e-12)


def island_basin(n: int, dx: float, seed: int, hump_amp: float = 0.5,
                 hump_radius: float = 20.0, island: bool = True,
                 min_sep: float | None = None):
    """Square basin (n x n cells, spacing dx): depth H = 20 - 18 D in [2, 20] m
    from 8 seeded Gaussians, minus an island Gaussian of height 24 m and width
    30 m (H <= 0 is dry land), and a Gaussian hump of the given amplitude on a
    wet point (depth >= 10 m) at least min_sep from the island centre
    (default: 100 m, or 0.3 of the side on smaller basins).  Returns (H, h0);
    the water is at rest."""
    rng = np.random.default_rng(seed)
    L = n * dx
    xc = centres(n, dx)
    D = gaussian_field(rng, n, n, L, L, xc, xc)
    H = 20.0 - 18.0 * D
    X, Y = np.meshgrid(xc, xc)
    ci = rng.uniform(0.25 * L, 0.75 * L, 2)
    if island:
        H = H - 24.0 * np.exp(-((X - ci[0]) ** 2 + (Y - ci[1]) ** 2) /
                              (2.0 * 30.0 ** 2))
    if hump_amp == 0.0:
        return H, np.where(H > 0.0, H, 0.0)
    sep = min(100.0, 0.3 * L) if min_sep is None else min_sep
    for _ in range(10000):
        ce = rng.uniform(0.1 * L, 0.9 * L, 2)
        i = min(int(ce[0] / dx), n - 1)
        j = min(int(ce[1] / dx), n - 1)
        far = math.hypot(ce[0] - ci[0], ce[1] - ci[1]) >= sep
        if H[j, i] >= 10.0 and (far or not island):
            break
    else:
        raise RuntimeError("no wet hump position found")
    eta0 = hump_amp * np.exp(-((X - ce[0]) ** 2 + (Y - ce[1]) ** 2) /
                             hump_radius ** 2)
    h0 = np.where(H > 0.0, H + eta0, 0.0)
    h0 = np.maximum(h0, 0.0)
    return H, h0


def case_c2(n: int = 512, steps: int = 1000, precision: str = "f64",
            seed: int = SEED_C2, island: bool = True) -> Case:
    """2D basin n x n (512 by default), dx = dy = 1 m, seeded bathymetry of
    depth 2-20 m with a dry island, Gaussian hump of 0.5 m / 20 m on wet water,
    zero velocity, walls.  island=False: the same basin without the island
    (fully wet)."""
    H, h0 = island_basin(n, 1.0, seed, island=island)
    z = np.zeros_like(h0)
    tol = 1e-10 if precision == "f64" else 1e-6
    c = Case("c2" if island else "c2-wet", n, n, 1.0, 1.0, H, h0, z,
             z.copy(), steps,
             precision=precision, solve_tol=tol, cfl=CFL_2D,
             dry_eps=1e-10 if precision == "f64" else 1e-5)
    rho = jacobi_radius_bound(float(h0.max()), c.dx, c.dy)
    c.omega = srj_schedule(rho, 64)
    c.check_every = 64
    return c


def case_dambreak(n: int = 1000, eps: float = 1e-5,
                  precision: str = "f64") -> Case:
    """The circular dam-break of Section 7.7, the workload of the paper's
    timings (Table 2): [-5, 5]^2 in n x n cells, still-water depth
    H = 1 - 0.25 exp(-x^2 - y^2), h0 = H inside r <= 0.5 and H + 0.25
    outside, at rest, CFL 0.9, open boundaries, t in [0, 1] s; eps is the
    stop tolerance of eq. (32).  `steps` is left 0: the run goes to t = 1."""
    dx = 10.0 / n
    xc = -5.0 + (np.arange(n) + 0.5) * dx
    X, Y = np.meshgrid(xc, xc)
    H = 1.0 - 0.25 * np.exp(-X * X - Y * Y)
    h0 = np.where(np.hypot(X, Y) <= 0.5, H, H + 0.25)
    z = np.zeros_like(h0)
    c = Case(f"dambreak{n}", n, n, dx, dx, H, h0, z, z.copy(), 0,
             precision=precision, solve_tol=eps, cfl=0.9,
             dry_eps=1e-10 if precision == "f64" else 1e-5, open_sides=15)
    rho = jacobi_radius_bound(float(h0.max()), c.dx, c.dy)
    c.omega = srj_schedule(rho, 64)
    c.check_every = 64
    return c


def case_c3(n: int = 2048, steps: int = 4000) -> Case:
    """Plane beach: n x n (2048 by default), dx = dy = 0.05 m, x in
    [0, n dx]; still-water depth 1 m for x < 70 m, slope 1:20 up to the
    shoreline at 90 m and beyond (dry land); y-invariant.  Solitary wave of
    eq. (33) with A = 0.3 m on H = 1 m centred at x = 50 m moving towards the
    beach; breaking terms on (B1 = 0.15, B2 = 0.5).  FP32 bulk."""
    dx = 0.05
    x = centres(n, dx)
    L = n * dx
    scale = L / 102.4
    x_toe, x_shore = 70.0 * scale, 90.0 * scale
    Hx = np.where(x < x_toe, 1.0, 1.0 - (x - x_toe) / 20.0)
    eta, u = solitary_wave(x, 0.3, 1.0, 50.0 * scale)
    hx = np.where(Hx > 0.0, np.maximum(Hx + eta, 0.0), 0.0)
    qx = hx * u
    H = np.tile(Hx, (n, 1))
    h = np.tile(hx, (n, 1))
    hu = np.tile(qx, (n, 1))
    c = Case("c3", n, n, dx, dx, H, h, hu, np.zeros_like(h), steps,
             breaking_on=1, precision="f32", solve_tol=1e-6, dry_eps=1e-5,
             cfl=CFL_2D)
    rho = jacobi_radius_bound(float(h.max()), dx, dx)
    c.omega = srj_schedule(rho, 64)
    c.check_every = 64
    del x_shore
    return c


C4_SIDES = (128, 256, 512, 768, 1024)


C4_SOURCE_SEP = 100.0   # m between the source and the island centre


def c4_has_island(n: int, dx: float = 1.0) -> bool:
    """Whether a basin of side n keeps the source C4_SOURCE_SEP from the
    island wherever the island falls: the island centre lies in
    [0.25 L, 0.75 L]^2 and the source in [0.1 L, 0.9 L]^2, so the farthest
    source point is at least 0.4 sqrt(2) L away."""
    return 0.4 * math.sqrt(2.0) * n * dx >= C4_SOURCE_SEP


def case_c4_member(k: int, seed: int = SEED_C4, sides=C4_SIDES,
                   steps: int = 500, precision: str = "f32",
                   island: bool | None = None) -> Case:
    """Scenario k of the ensemble workload, drawn from its own generator
    (seed + k): side n uniform over `sides`, the basin of c2 at that side
    (dx = 1 m), a Gaussian source of amplitude U[0.1, 1] m and radius 20 m
    on wet water at least 100 m from the island centre.  Sides too small for
    that separation (c4_has_island) get the basin without the island: a
    source of up to 1 m next to the island's near-vertical flanks drives
    thin films on the dry slope to velocities that collapse the time step,
    in the FP64 oracle as on the GPU.  island=True/False overrides the rule
    (the separation then falls back to 0.3 of the side).  FP32 bulk unless
    precision says otherwise."""
    rng = np.random.default_rng(seed + k)
    n = int(sides[int(rng.integers(len(sides)))])
    amp = float(rng.uniform(0.1, 1.0))
    basin_seed = int(rng.integers(1 << 31))
    if island is None:
        isl, sep = c4_has_island(n), C4_SOURCE_SEP
    else:
        isl, sep = island, None
    H, h0 = island_basin(n, 1.0, basin_seed, hump_amp=amp, hump_radius=20.0,
                         island=isl, min_sep=sep)
    z = np.zeros_like(h0)
    f32 = precision == "f32"
    c = Case(f"c4-{k}", n, n, 1.0, 1.0, H, h0, z, z.copy(), steps,
             precision=precision, solve_tol=1e-6 if f32 else 1e-10,
             dry_eps=1e-5 if f32 else 1e-10, cfl=CFL_2D)
    rho = jacobi_radius_bound(float(h0.max()), c.dx, c.dy)
    c.omega = srj_schedule(rho, 64)
    c.check_every = 64
    return c


def case_c4(members: int = 64, seed: int = SEED_C4, sides=C4_SIDES,
            steps: int = 500, precision: str = "f32") -> list:
    """Ensemble workload: `members` independent scenarios (case_c4_member),
    64 by default, of uneven sizes (expected total about 25.4 M cells)."""
    return [case_c4_member(k, seed, sides, steps, precision)
            for k in range(members)]


def c5_initial_surface(n: int, dx: float, seed: int, amp: float = 0.5,
                       radius: float = 100.0) -> np.ndarray:
    """A Gaussian surface bump of the given amplitude and radius [m] at a
    seeded position in the central half of the domain."""
    rng = np.random.default_rng(seed)
    L = n * dx
    c = rng.uniform(0.25 * L, 0.75 * L, 2)
    xc = centres(n, dx)
    X, Y = np.meshgrid(xc, xc)
    return amp * np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2) / radius ** 2)


def case_c5(n: int = 1024, steps: int = 2000, precision: str = "f32",
            seed: int = SEED_C5, dx: float = 10.0, cfl_dt: float = 0.5):
    """Adjoint workload: n x n (1024 by default) fully wet basin, dx = dy =
    10 m, depth H = 5 + 45 D in [5, 50] m from 8 seeded Gaussians, initial
    surface a 0.5 m bump of radius 100 m at a seeded position, at rest.  The
    time step is fixed: cfl_dt / max((|u|+c)/dx + (|v|+c)/dy) of the initial
    state (below the 2D limit of 0.7 through the run).  16 seeded gauge cells
    in the interior.  Returns (Case with fixed dt, eta0, gauges, target_eta0)
    where target_eta0 is the initial surface of the seeded target run
    (another position, amplitude U[0.25, 0.75] m)."""
    rng = np.random.default_rng(seed)
    xc = centres(n, dx)
    L = n * dx
    D = gaussian_field(rng, n, n, L, L, xc, xc)
    H = 5.0 + 45.0 * D
    eta0 = c5_initial_surface(n, dx, seed + 1)
    amp_t = float(np.random.default_rng(seed + 1000).uniform(0.25, 0.75))
    target_eta0 = c5_initial_surface(n, dx, seed + 1000, amp=amp_t)
    g_rng = np.random.default_rng(seed + 7)
    gi = g_rng.integers(n // 10, n - n // 10, size=(16, 2))
    gauges = gi[:, 1] * n + gi[:, 0]
    h0 = H + eta0
    z = np.zeros_like(h0)
    lam = 2.0 * float(np.sqrt(G * h0.max())) / dx
    dt = cfl_dt / lam
    f32 = precision == "f32"
    c = Case("c5", n, n, dx, dx, H, h0, z, z.copy(), steps, precision=precision,
             solve_tol=1e-6 if f32 else 1e-10, dry_eps=1e-5 if f32 else 1e-10,
             cfl=CFL_2D)
    rho = jacobi_radius_bound(float(h0.max()), dx, dx)
    c.omega = srj_schedule(rho, 64)
    c.check_every = 64
    c.fixed_dt = 1
    c.dt_fixed = dt
    return c, eta0, gauges, target_eta0


def synthetic_gauge_record(case, gauges, steps: int, seed: int = SEED_C5):
    """A seeded gauge record (steps x ngauges): the still-water depth at each
    gauge plus a few centimetres of smooth seeded oscillation, a target for
    the misfit that is independent of any solver run."""
    rng = np.random.default_rng(seed + 2000)
    t = case.dt_fixed * np.arange(1, steps + 1)[:, None]
    a = rng.uniform(0.01, 0.05, size=(1, len(gauges)))
    w = rng.uniform(0.02, 0.2, size=(1, len(gauges)))
    ph = rng.uniform(0.0, 2 * np.pi, size=(1, len(gauges)))
    return case.H.reshape(-1)[gauges][None, :] + a * np.sin(w * t + ph)


def lake_at_rest(n: int = 64, dx: float = 1.0, seed: int = SEED_C2,
                 island: bool = True) -> Case:
    """The c2 geometry with the hump removed (still water, surface 0)."""
    H, _ = island_basin(n, dx, seed, hump_amp=0.0, island=island)
    h0 = np.where(H > 0.0, H, 0.0)
    z = np.zeros_like(h0)
    c = Case("lake", n, n, dx, dx, H, h0, z, z.copy(), 100, cfl=CFL_2D)
    return c


def random_wet_state(rng: np.random.Generator, nx: int, ny: int, dx: float,
                     dy: float, depth=(2.0, 6.0), amp: float = 0.3,
                     vel: float = 0.5):
    """A smooth random fully wet state (for component checks): bathymetry,
    depth, discharges."""
    xc, yc = centres(nx, dx), centres(ny, dy)
    D = gaussian_field(rng, nx, ny, nx * dx, ny * dy, xc, yc, 4)
    H = depth[0] + (depth[1] - depth[0]) * D
    E = gaussian_field(rng, nx, ny, nx * dx, ny * dy, xc, yc, 4)
    h = H + amp * (E - 0.5)
    U = gaussian_field(rng, nx, ny, nx * dx, ny * dy, xc, yc, 3)
    V = gaussian_field(rng, nx, ny, nx * dx, ny * dy, xc, yc, 3)
    hu = h * vel * (U - 0.5)
    hv = h * vel * (V - 0.5)
    return H, h, hu, hv
