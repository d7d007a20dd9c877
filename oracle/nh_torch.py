"""Differentiable FP64 CPU oracle of the 2D time step (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU baseline use this
module; the product path never does.

A second, independent statement of the 2D scheme, written with plain PyTorch
CPU tensor operations in float64 so that torch's automatic differentiation
gives the exact derivatives of the discrete step:
  * reverse mode (``torch.autograd``): the adjoint, i.e. gradients of a misfit
    with respect to the initial surface and the bathymetry;
  * forward mode (``torch.func.jvp``): the tangent-linear model.
It follows the same readings of the paper as the C oracle (``nh_oracle.c``),
but states the pressure step differently: instead of the closed-form
five-point rows it imposes the literal constraint at every corner --
eq. (37), with the discharges and w corrected by eq. (36) and (41) -- and
solves the resulting affine system for the corner pressures with a dense
direct solve (``torch.linalg.solve``).  It is therefore meant for small grids
(a few thousand corners).  Walls on every side, no breaking terms.

Sections and equations cited are those of Escalante, Morales de Luna &
Castro (arXiv 1706.04551).
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

DT = torch.float64


@dataclass
class TorchParams:
    nx: int
    ny: int
    dx: float
    dy: float
    dt: float                # fixed time step of every step
    g: float = 9.81
    delta: float = 1e-5      # desingularisation depth (Section 4.5)
    dry_eps: float = 1e-10   # h <= dry_eps is dry
    nh_on: bool = True
    manning: float = 0.0     # Gauckler-Manning n of the friction law (Section 2)


# --------------------------------------------------------------------------
# ghosts: walls by mirror images, two ghost layers (Section 4.1 stencil)
# --------------------------------------------------------------------------
def pad_cells(a: torch.Tensor, px: float, py: float) -> torch.Tensor:
    """[ny, nx] -> [ny+4, nx+4]; ghost -1 mirrors cell 0, -2 mirrors cell 1;
    px, py = +1 (even) or -1 (odd) parity across the x / y walls."""
    a = torch.cat([px * a[:, 1:2], px * a[:, 0:1], a,
                   px * a[:, -1:], px * a[:, -2:-1]], dim=1)
    a = torch.cat([py * a[1:2, :], py * a[0:1, :], a,
                   py * a[-1:, :], py * a[-2:-1, :]], dim=0)
    return a


def pad_corners(p: torch.Tensor) -> torch.Tensor:
    """[..., ny+1, nx+1] -> [..., ny+3, nx+3] reflected about the wall corner
    rows (p at corner -1 equals p at corner 1)."""
    p = torch.cat([p[..., :, 1:2], p, p[..., :, -2:-1]], dim=-1)
    p = torch.cat([p[..., 1:2, :], p, p[..., -2:-1, :]], dim=-2)
    return p


# --------------------------------------------------------------------------
# Section 4.1 / 4.5 building blocks, elementwise
# --------------------------------------------------------------------------
def desing(h, q, delta):
    """u = sqrt(2) h q / sqrt(h^4 + max(h^4, delta^4)) (Section 4.5)."""
    h4 = h ** 4
    return (2.0 ** 0.5) * h * q / torch.sqrt(h4 + torch.clamp(h4, min=delta ** 4))


def minmod(a, b):
    zero = torch.zeros_like(a)
    return torch.where((a > 0) & (b > 0), torch.minimum(a, b),
                       torch.where((a < 0) & (b < 0), torch.maximum(a, b), zero))


def reconstruct(hm, h0, hp, em, e0, ep, um, u0, up, vm, v0, vp, dry_eps):
    """MUSCL-minmod values of the middle cell at its minus-side (L) and
    plus-side (R) edge; eta and velocity slopes vanish next to a dry cell."""
    sh = minmod(hp - h0, h0 - hm)
    wet = (hm > dry_eps) & (h0 > dry_eps) & (hp > dry_eps)
    zero = torch.zeros_like(h0)
    se = torch.where(wet, minmod(ep - e0, e0 - em), zero)
    su = torch.where(wet, minmod(up - u0, u0 - um), zero)
    sv = torch.where(wet, minmod(vp - v0, v0 - vm), zero)
    R = {"h": h0 + 0.5 * sh, "eta": e0 + 0.5 * se, "un": u0 + 0.5 * su,
         "ut": v0 + 0.5 * sv}
    L = {"h": h0 - 0.5 * sh, "eta": e0 - 0.5 * se, "un": u0 - 0.5 * su,
         "ut": v0 - 0.5 * sv}
    for F in (L, R):
        F["qn"] = F["h"] * F["un"]
        F["qt"] = F["h"] * F["ut"]
        F["H"] = F["h"] - F["eta"]
    return L, R


def pvm(L, R, g, dry_eps):
    """PVM-HLL fluctuations (eq. 18-19, Roe average of Section 4.1) between the
    left state L and the right state R, normal components (h, qn, qt)."""
    he = 0.5 * (L["h"] + R["h"])
    sL, sR = torch.sqrt(L["h"]), torch.sqrt(R["h"])
    both_dry = (L["h"] <= dry_eps) & (R["h"] <= dry_eps)
    den = torch.where(both_dry, torch.ones_like(sL), sL + sR)
    ue = (L["un"] * sL + R["un"] * sR) / den
    ce = torch.sqrt(g * he)
    SL = torch.minimum(ue - ce, L["un"] - torch.sqrt(g * L["h"]))
    SR = torch.maximum(ue + ce, R["un"] + torch.sqrt(g * R["h"]))
    ok = (SR - SL > 0) & ~both_dry
    dS = torch.where(ok, SR - SL, torch.ones_like(SR))
    a0 = (SR * torch.abs(SL) - SL * torch.abs(SR)) / dS
    a1 = (torch.abs(SR) - torch.abs(SL)) / dS
    deta = R["eta"] - L["eta"]
    deta = torch.where((R["h"] <= dry_eps) & (L["eta"] < -R["H"]),
                       torch.zeros_like(deta), deta)
    deta = torch.where((L["h"] <= dry_eps) & (R["eta"] < -L["H"]),
                       torch.zeros_like(deta), deta)
    Rv = [R["qn"] - L["qn"],
          (R["qn"] * R["un"] - L["qn"] * L["un"]) + g * he * deta,
          R["qn"] * R["ut"] - L["qn"] * L["ut"]]
    dU = [deta, R["qn"] - L["qn"], R["qt"] - L["qt"]]
    zero = torch.zeros_like(he)
    Dm = [torch.where(ok, 0.5 * ((1 - a1) * Rv[m] - a0 * dU[m]), zero)
          for m in range(3)]
    Dp = [torch.where(ok, 0.5 * ((1 + a1) * Rv[m] + a0 * dU[m]), zero)
          for m in range(3)]
    return Dm, Dp


def interior(L, R, h0, g):
    """Volume term of eq. (22) in its mid-point form (eq. 30)."""
    return [R["qn"] - L["qn"],
            (R["qn"] * R["un"] - L["qn"] * L["un"]) + g * h0 * (R["eta"] - L["eta"]),
            R["qn"] * R["ut"] - L["qn"] * L["ut"]]


# --------------------------------------------------------------------------
# one finite-volume stage (eq. 20-22, 30), 2D dimension-wise
# --------------------------------------------------------------------------
def fv_stage(P: TorchParams, h, q1, q2, H, dt):
    g, eps, de = P.g, P.dry_eps, P.delta
    hp = pad_cells(h, 1.0, 1.0)
    Hp = pad_cells(H, 1.0, 1.0)
    q1p = pad_cells(q1, -1.0, 1.0)
    q2p = pad_cells(q2, 1.0, -1.0)
    u = desing(hp, q1p, de)
    v = desing(hp, q2p, de)
    eta = hp - Hp
    ny, nx = h.shape

    def faces(axis):
        # faces of the cells -1 .. n along `axis`, interior range across it
        if axis == 1:   # x: rows 2..ny+1 of the padded array
            sl = lambda a, s: a[2:ny + 2, 1 + s:nx + 3 + s]  # noqa: E731
            un, ut = u, v
        else:
            sl = lambda a, s: a[1 + s:ny + 3 + s, 2:nx + 2]  # noqa: E731
            un, ut = v, u
        return reconstruct(sl(hp, -1), sl(hp, 0), sl(hp, 1),
                           sl(eta, -1), sl(eta, 0), sl(eta, 1),
                           sl(un, -1), sl(un, 0), sl(un, 1),
                           sl(ut, -1), sl(ut, 0), sl(ut, 1), eps)

    def sweep(axis):
        L, R = faces(axis)   # index 0 <-> cell -1, 1 <-> cell 0, ...
        if axis == 1:
            take = lambda F, s: {k: v[:, 1 + s:nx + 1 + s] for k, v in F.items()}  # noqa: E731
        else:
            take = lambda F, s: {k: v[1 + s:ny + 1 + s, :] for k, v in F.items()}  # noqa: E731
        Dm_e, _ = pvm(take(R, 0), take(L, 1), g, eps)
        _, Dp_w = pvm(take(R, -1), take(L, 0), g, eps)
        I = interior(take(L, 0), take(R, 0), h, g)
        return [(Dm_e[m] + Dp_w[m]) + I[m] for m in range(3)]

    fx = sweep(1)
    fy = sweep(0)
    hs = h - dt * (fx[0] / P.dx + fy[0] / P.dy)
    q1s = q1 - dt * (fx[1] / P.dx + fy[2] / P.dy)
    q2s = q2 - dt * (fx[2] / P.dx + fy[1] / P.dy)
    hs = torch.clamp(hs, min=0.0)
    dry = hs <= eps
    q1s = torch.where(dry, torch.zeros_like(q1s), q1s)
    q2s = torch.where(dry, torch.zeros_like(q2s), q2s)
    return hs, q1s, q2s


# --------------------------------------------------------------------------
# non-hydrostatic step: literal constraint at the corners, dense solve
# --------------------------------------------------------------------------
class Corrector:
    """Cell quantities of one stage needed by the correction (eq. 36) and by
    the constraint (eq. 37): padded h, zeta = h - 2H and their centred
    slopes, for the cells -1 .. n in both directions."""

    def __init__(self, P: TorchParams, h, H):
        self.P = P
        ny, nx = h.shape
        hp = pad_cells(h, 1.0, 1.0)
        zp = hp - 2.0 * pad_cells(H, 1.0, 1.0)
        # cells -1..nx (x) and -1..ny (y): padded index 1..n+2
        self.h = hp[1:ny + 3, 1:nx + 3]
        self.zeta = zp[1:ny + 3, 1:nx + 3]
        self.zx = (zp[1:ny + 3, 2:nx + 4] - zp[1:ny + 3, 0:nx + 2]) / (2.0 * P.dx)
        self.zy = (zp[2:ny + 4, 1:nx + 3] - zp[0:ny + 2, 1:nx + 3]) / (2.0 * P.dy)

    def T(self, p):
        """T^Hor_N, T^Hor_S, T^Ver_E, T^Ver_W (Appendix A.2) of the cells
        -1..n for corner pressures p [..., ny+1, nx+1]."""
        P = self.P
        pp = pad_corners(p)          # corner k <-> index k + 1
        ny1, nx1 = self.h.shape      # ny + 2, nx + 2 (cells -1..n)
        # corners (i, j) of cell i in -1..n: padded corner index i + 1
        c = lambda di, dj: pp[..., dj:dj + ny1, di:di + nx1]  # noqa: E731
        pSW, pSE, pNW, pNE = c(0, 0), c(1, 0), c(0, 1), c(1, 1)
        h, zx, zy = self.h, self.zx, self.zy
        TN = -0.5 * h * (pNE - pNW) / P.dx - 0.5 * ((pNE + pNW) / 2.0) * zx
        TS = -0.5 * h * (pSE - pSW) / P.dx - 0.5 * ((pSE + pSW) / 2.0) * zx
        TE = -0.5 * h * (pNE - pSE) / P.dy - 0.5 * ((pNE + pSE) / 2.0) * zy
        TW = -0.5 * h * (pNW - pSW) / P.dy - 0.5 * ((pNW + pSW) / 2.0) * zy
        return TN, TS, TE, TW


def constraint(P: TorchParams, C: Corrector, q1, q2, w, p, dt):
    """Eq. (37) at every corner with the corrected discharges (eq. 36) and the
    corrected w (eq. 41): h_c div q - q . grad(zeta) + 2 (h_c w + dt p), for
    corner pressures p [..., ny+1, nx+1] (batched)."""
    ny, nx = q1.shape
    q1p = pad_cells(q1, -1.0, 1.0)[1:ny + 3, 1:nx + 3]
    q2p = pad_cells(q2, 1.0, -1.0)[1:ny + 3, 1:nx + 3]
    TN, TS, TE, TW = C.T(p)
    # corner (k, l) has the cells SW=(k-1,l-1) SE=(k,l-1) NW=(k-1,l) NE=(k,l);
    # in the -1..n cell arrays cell i sits at index i + 1
    cell = lambda a, di, dj: a[..., dj:dj + ny + 1, di:di + nx + 1]  # noqa: E731
    SW, SE, NW, NE = (0, 0), (1, 0), (0, 1), (1, 1)
    half_dt = 0.5 * dt
    q1E = 0.5 * (cell(q1p, *NE) + cell(q1p, *SE)) + half_dt * cell(TS, *NE) + half_dt * cell(TN, *SE)
    q1W = 0.5 * (cell(q1p, *NW) + cell(q1p, *SW)) + half_dt * cell(TS, *NW) + half_dt * cell(TN, *SW)
    q2N = 0.5 * (cell(q2p, *NE) + cell(q2p, *NW)) + half_dt * cell(TW, *NE) + half_dt * cell(TE, *NW)
    q2S = 0.5 * (cell(q2p, *SE) + cell(q2p, *SW)) + half_dt * cell(TW, *SE) + half_dt * cell(TE, *SW)
    z = C.zeta
    zE = 0.5 * (cell(z, *NE) + cell(z, *SE))
    zW = 0.5 * (cell(z, *NW) + cell(z, *SW))
    zN = 0.5 * (cell(z, *NE) + cell(z, *NW))
    zS = 0.5 * (cell(z, *SE) + cell(z, *SW))
    hh = C.h
    hc = 0.25 * (cell(hh, *SW) + cell(hh, *SE) + cell(hh, *NW) + cell(hh, *NE))
    divQ = (q1E - q1W) / P.dx + (q2N - q2S) / P.dy
    Qx = (q1E + q1W) / 2.0
    Qy = (q2N + q2S) / 2.0
    gzx = (zE - zW) / P.dx
    gzy = (zN - zS) / P.dy
    return hc * divQ - (Qx * gzx + Qy * gzy) + 2.0 * (hc * w + dt * p)


def solve_pressure(P: TorchParams, C: Corrector, q1, q2, w, dt):
    """The corner pressures that make the constraint vanish: it is affine in
    p, c(p) = c(0) + M p, with M probed column by column (unit vectors)."""
    ny, nx = q1.shape
    n = (nx + 1) * (ny + 1)
    zero = torch.zeros((ny + 1, nx + 1), dtype=DT)
    c0 = constraint(P, C, q1, q2, w, zero, dt).reshape(n)
    E = torch.eye(n, dtype=DT).reshape(n, ny + 1, nx + 1)
    M = (constraint(P, C, q1, q2, w, E, dt).reshape(n, n) - c0[None, :]).T
    return torch.linalg.solve(M, -c0).reshape(ny + 1, nx + 1)


def correct(P: TorchParams, C: Corrector, hs, q1s, q2s, w, p, dt):
    """Correction of the discharges (eq. 36) and of w (eq. 41) with the
    desingularised division by h_c (Section 4.5)."""
    ny, nx = hs.shape
    TN, TS, TE, TW = C.T(p)
    inner = lambda a: a[1:ny + 1, 1:nx + 1]  # noqa: E731
    q1 = q1s + dt * (0.5 * (inner(TN) + inner(TS)))
    q2 = q2s + dt * (0.5 * (inner(TE) + inner(TW)))
    dry = hs <= P.dry_eps
    q1 = torch.where(dry, torch.zeros_like(q1), q1)
    q2 = torch.where(dry, torch.zeros_like(q2), q2)
    hh = C.h
    cell = lambda a, di, dj: a[dj:dj + ny + 1, di:di + nx + 1]  # noqa: E731
    hc = 0.25 * (cell(hh, 0, 0) + cell(hh, 1, 0) + cell(hh, 0, 1) + cell(hh, 1, 1))
    w_new = w + dt * desing(hc, p, P.delta)
    return q1, q2, w_new


def friction(P: TorchParams, hs, q1s, q2s, dt):
    """Manning friction of Section 2, semi-implicit on the stage's
    finite-volume result, in wet cells: q / (1 + dt g n^2 |u| / h^(4/3)),
    |u| from the desingularised velocities.  |u| has derivative 0 at 0 (the
    convention of the GPU adjoint for the norm's kink)."""
    wet = hs > P.dry_eps
    hw = torch.where(wet, hs, torch.ones_like(hs))
    u, v = desing(hw, q1s, P.delta), desing(hw, q2s, P.delta)
    s2 = u * u + v * v
    pos = s2 > 0
    speed = torch.where(pos, torch.sqrt(torch.where(pos, s2,
                                                     torch.ones_like(s2))),
                        torch.zeros_like(s2))
    den = 1.0 + dt * P.g * P.manning ** 2 * speed / (hw * hw ** (1.0 / 3.0))
    return (torch.where(wet, q1s / den, q1s),
            torch.where(wet, q2s / den, q2s))


def stage(P: TorchParams, h, q1, q2, w, H, dt):
    hs, q1s, q2s = fv_stage(P, h, q1, q2, H, dt)
    if P.manning > 0:
        q1s, q2s = friction(P, hs, q1s, q2s, dt)
    if not P.nh_on:
        return hs, q1s, q2s, w, None
    C = Corrector(P, hs, H)
    p = solve_pressure(P, C, q1s, q2s, w, dt)
    q1n, q2n, wn = correct(P, C, hs, q1s, q2s, w, p, dt)
    return hs, q1n, q2n, wn, p


def step(P: TorchParams, h, q1, q2, w, H):
    """TVD-RK2 (Heun) step of Section 6 with the fixed dt P.dt."""
    dt = P.dt
    h1, q11, q21, w1, _ = stage(P, h, q1, q2, w, H, dt)
    h2, q12, q22, w2, p2 = stage(P, h1, q11, q21, w1, H, dt)
    return (0.5 * (h + h2), 0.5 * (q1 + q12), 0.5 * (q2 + q22),
            0.5 * (w + w2), p2)


# --------------------------------------------------------------------------
# gauge misfit and its derivatives
# --------------------------------------------------------------------------
def misfit(P: TorchParams, eta0, H, gauges, target, nsteps: int):
    """J = 1/2 sum_{n=1..nsteps} sum_g (h^n_g - target[n-1, g])^2 for the run
    from h0 = max(H + eta0, 0), zero discharge, w = 0.
    gauges: flat cell indices (j * nx + i); target [nsteps, ngauges]."""
    h = torch.clamp(H + eta0, min=0.0)
    q1 = torch.zeros_like(h)
    q2 = torch.zeros_like(h)
    w = torch.zeros((P.ny + 1, P.nx + 1), dtype=DT)
    gi = torch.as_tensor(gauges, dtype=torch.long)
    tg = torch.as_tensor(target, dtype=DT)
    J = torch.zeros((), dtype=DT)
    for n in range(nsteps):
        h, q1, q2, w, _ = step(P, h, q1, q2, w, H)
        r = h.reshape(-1)[gi] - tg[n]
        J = J + 0.5 * torch.sum(r * r)
    return J


def gradient(P: TorchParams, eta0, H, gauges, target, nsteps: int):
    """(J, dJ/deta0 at fixed H, dJ/dH at fixed eta0) by reverse mode."""
    e = torch.as_tensor(eta0, dtype=DT).clone().requires_grad_(True)
    b = torch.as_tensor(H, dtype=DT).clone().requires_grad_(True)
    J = misfit(P, e, b, gauges, target, nsteps)
    ge, gb = torch.autograd.grad(J, (e, b))
    return float(J.detach()), ge.numpy(), gb.numpy()


def tangent(P: TorchParams, eta0, H, d_eta0, d_H, gauges, target,
            nsteps: int):
    """(J, dJ) with dJ the derivative of J along (d_eta0, d_H) by forward
    mode (the tangent-linear model)."""
    from torch.func import jvp
    e = torch.as_tensor(eta0, dtype=DT)
    b = torch.as_tensor(H, dtype=DT)
    de = torch.as_tensor(d_eta0, dtype=DT)
    db = torch.as_tensor(d_H, dtype=DT)
    J, dJ = jvp(lambda x, y: misfit(P, x, y, gauges, target, nsteps),
                (e, b), (de, db))
    return float(J), float(dJ)


def run(P: TorchParams, h, q1, q2, H, nsteps: int, w=None):
    """Plain forward run (no gradients): state after nsteps."""
    with torch.no_grad():
        h = torch.as_tensor(h, dtype=DT)
        q1 = torch.as_tensor(q1, dtype=DT)
        q2 = torch.as_tensor(q2, dtype=DT)
        Ht = torch.as_tensor(H, dtype=DT)
        w = (torch.zeros((P.ny + 1, P.nx + 1), dtype=DT) if w is None
             else torch.as_tensor(w, dtype=DT))
        p = None
        for _ in range(nsteps):
            h, q1, q2, w, p = step(P, h, q1, q2, w, Ht)
        return {"h": h.numpy(), "hu": q1.numpy(), "hv": q2.numpy(),
                "w": w.numpy(), "p": None if p is None else p.numpy()}
