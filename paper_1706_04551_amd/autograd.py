"""torch.autograd.Function over the adjoint of the time stepper.

``AdjointRun.apply(eta0, H, solver, gauges, target, nsteps, ckpt_every,
adj_tol)`` runs the solver from h0 = max(H + eta0, 0) at rest for nsteps
fixed-dt steps and returns the gauge misfit J (include/nhswe.h,
nh_adjoint_run); its backward gives dJ/deta0 and dJ/dH (at fixed eta0).  The
library computes J and both gradients in one call (forward run, then the
adjoint run back through checkpointed segments), so the gradients are kept
from the forward call.
"""
from __future__ import annotations

import numpy as np
import torch


class AdjointRun(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eta0, H, solver, gauges, target, nsteps, ckpt_every=100,
                adj_tol=1e-8):
        e = eta0.detach().cpu().numpy().astype(np.float64)
        b = H.detach().cpu().numpy().astype(np.float64)
        h0 = np.maximum(b + e, 0.0)
        z = np.zeros_like(h0)
        solver.set_bathymetry(b)
        solver.set_state(h0, z, z)
        r = solver.adjoint(nsteps, gauges, target, ckpt_every, adj_tol)
        wet = (b + e > 0.0).astype(np.float64)
        # results live where the inputs do (autograd requires gradients on
        # the device and in the dtype of their inputs)
        g_eta = torch.from_numpy(r["dh0"] * wet).to(device=eta0.device,
                                                    dtype=eta0.dtype)
        g_H = torch.from_numpy(r["dH"] + r["dh0"] * wet).to(device=H.device,
                                                           dtype=H.dtype)
        ctx.save_for_backward(g_eta, g_H)
        return torch.tensor(r["J"], dtype=torch.float64, device=eta0.device)

    @staticmethod
    def backward(ctx, gJ):
        g_eta, g_H = ctx.saved_tensors
        return ((gJ.to(g_eta.dtype) * g_eta), (gJ.to(g_H.dtype) * g_H),
                None, None, None, None, None, None)
