"""Gradient of the time-integrated penalization force through the HIP adjoint.

J(theta, dus) = sum_{n=1..N} dt F_x(U^n, t^n), with U^n from N RK4 steps of
fixed size dt on a frozen grid, F_x the x-component of the penalization force
(Sec. 2.2, midpoint rule), theta = (amp, freq, phase) the pitch parameters of
the plate mask and dus a static extra solid velocity.  The forward pass keeps
one checkpoint per RK4 step: the interiors of the active blocks of the step's
input (the adjoint step re-synchronises ghost layers itself, and unused pool
slots are never read).  The backward pass scatters each checkpoint back into
a scratch pool and runs the library's hand-written adjoint
(wacm_rk4_step_adj, wacm_force_adj) from the last step to the first.  Every
step of both passes runs in libwacm.
"""
from __future__ import annotations

import torch

from . import wacm


def _params(base: dict, theta) -> dict:
    p = dict(base)
    p["amp"], p["freq"], p["phase"] = (float(v) for v in theta)
    return p


class ForceObjective(torch.autograd.Function):
    """J = ForceObjective.apply(theta, dus, grid, params, U0, dt, nsteps).

    theta: float64 tensor (3,) on the CPU; dus: pool-dtype CUDA tensor
    (capacity, 3, bs^3); U0: initial pool (not modified).  Returns a float64
    0-d CUDA tensor.  Gradients flow to theta and dus."""

    @staticmethod
    def forward(ctx, theta, dus, grid: wacm.Grid, params: dict, U0, dt: float, nsteps: int):
        prm = _params(params, theta.detach().cpu().tolist())
        U = U0.clone()
        work = grid.work()
        t_dev = torch.zeros(1, dtype=torch.float64, device=U.device)
        dt_dev = torch.full((1,), float(dt), dtype=torch.float64, device=U.device)
        out = torch.zeros(10, dtype=torch.float64, device=U.device)
        J = torch.zeros((), dtype=torch.float64, device=U.device)
        slots = torch.as_tensor(grid.info()[0], dtype=torch.int64, device=U.device)
        I = slice(grid.ng, grid.ng + grid.bs)
        ck = []
        for n in range(nsteps):
            ck.append(U[:, :, I, I, I].index_select(0, slots))
            t_dev.fill_(n * dt)
            grid.rk4_step(prm, t_dev, dt_dev, U, work, dus, dt_mode=wacm.DT_FIXED)
            grid.diagnostics(prm, (n + 1) * dt, U, out, dus)
            J += dt * out[5]
        ctx.grid, ctx.prm, ctx.dt, ctx.nsteps = grid, prm, float(dt), int(nsteps)
        ctx.ck, ctx.slots = ck, slots
        ctx.save_for_backward(dus, U)
        return J

    @staticmethod
    def backward(ctx, gJ):
        dus, UN = ctx.saved_tensors
        g, prm, dt, N = ctx.grid, ctx.prm, ctx.dt, ctx.nsteps
        lam = torch.zeros_like(UN)
        dth = torch.zeros(3, dtype=torch.float64, device=UN.device)
        dusbar = torch.zeros((g.capacity, 3, g.bs ** 3), dtype=torch.float64, device=UN.device)
        awork = g.adj_work()
        Un = torch.zeros_like(UN)  # scratch pool for the checkpoints
        I = slice(g.ng, g.ng + g.bs)
        g.force_adj(prm, N * dt, dt, UN, lam, dth, dusbar, dus)
        for n in range(N - 1, -1, -1):
            Un[:, :, I, I, I].index_copy_(0, ctx.slots, ctx.ck[n])
            g.rk4_step_adj(prm, n * dt, dt, Un, lam, dth, dusbar, dus, awork)
            if n >= 1:
                g.force_adj(prm, n * dt, dt, Un, lam, dth, dusbar, dus)
        ctx.ck = None
        gth = (gJ * dth).cpu()
        gdus = (gJ * dusbar).to(dus.dtype) if dus is not None else None
        return gth, gdus, None, None, None, None, None
