"""Gradients of the lesion-temperature loss through the coupled time steps, as a
``torch.autograd.Function`` whose forward and backward run in the native library.

Forward: ``steps`` coupled steps from the initial state, keeping (T, V) every
``checkpoint_every`` steps, then L = sum over the loss nodes of (T^N - T*)^2.
Backward: for each checkpoint segment, last first, recompute the segment's states from
its checkpoint, then run ``rafem_step_vjp`` from the segment's last step to its first,
accumulating dL/dk_e and dL/dw_e.  Steps are deterministic, so the recomputed states are
bitwise the forward states.  Each reverse step's adjoint solves start from the adjoint
states of the step after it (``phys.extrapolate`` 1; 2 on the sweep's first call), as the
forward solves start from the previous states.
"""
from __future__ import annotations

import torch

from . import _lib as rafem
from .sim import DeviceProblem


class _LesionLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, k_e, perf_e, dp: DeviceProblem, steps: int, every: int, tol: float,
                precision: str):
        dp.set_params(k_e.detach(), perf_e.detach())
        dp.reset()
        ckpt = {0: (dp.T.clone(), dp.V.clone())}
        for n in range(1, steps + 1):
            dp.step(tol, precision)
            if n % every == 0 and n < steps:
                ckpt[n] = (dp.T.clone(), dp.V.clone())
        loss = rafem.lesion_loss(dp.mesh, dp.loss_ids, dp.T_target, dp.T)
        ctx.T_final = dp.T.clone()
        ctx.dp, ctx.steps, ctx.every, ctx.tol, ctx.precision = dp, steps, every, tol, precision
        ctx.ckpt = ckpt
        return loss[0]

    @staticmethod
    def backward(ctx, gL):
        dp, steps, every, tol = ctx.dp, ctx.steps, ctx.every, ctx.tol
        mesh, p = dp.mesh, dp.phys
        lam = torch.zeros(mesh.n_nodes, dtype=torch.float64, device=dp.dev)
        # seed: dL/dT^N, scaled by the incoming gradient
        starts = sorted(ctx.ckpt)
        rafem.lesion_loss(mesh, dp.loss_ids, dp.T_target, ctx.T_final, scale=float(gL), grad=lam)
        gk = torch.zeros(mesh.n_elems, dtype=torch.float64, device=dp.dev)
        gw = torch.zeros_like(gk)
        p.reuse_bioheat = 1
        first = True
        for s0 in reversed(starts):
            s1 = min(s0 + every, steps)
            dp.restore(*ctx.ckpt[s0])
            Ts, Vs = [dp.T.clone()], [dp.V.clone()]
            for _ in range(s0, s1):
                dp.step(tol, ctx.precision)
                Ts.append(dp.T.clone())
                Vs.append(dp.V.clone())
            for j in range(s1 - s0, 0, -1):
                p.extrapolate = 2 if first else 1
                first = False
                rafem.step_vjp(mesh, p, dp.k_e, dp.perf_e, dp.sigma0_e, dp.dir_V, dp.dir_T,
                               Ts[j - 1], Vs[j], Ts[j], lam, gk, gw, tol=tol,
                               precision=ctx.precision)
        return gk, gw, None, None, None, None, None


def lesion_loss(dp: DeviceProblem, k_e: torch.Tensor, perf_e: torch.Tensor, steps: int,
                checkpoint_every: int = 10, tol: float = 1e-13, precision: str = "fp64"):
    """Differentiable loss: L(k_e, perf_e) after ``steps`` coupled steps of ``dp``'s problem."""
    if dp.loss_ids is None:
        raise ValueError("the problem has no loss region")
    return _LesionLoss.apply(k_e, perf_e, dp, int(steps), int(checkpoint_every), float(tol),
                             precision)


def fd_directional(dp: DeviceProblem, k_e, perf_e, dk, dw, h: float, steps: int,
                   tol: float = 1e-14, precision: str = "fp64") -> float:
    """Central finite difference of the lesion loss along (dk, dw) (host arrays of element
    values) with step h: (L(theta + h d) - L(theta - h d)) / (2 h), both forward runs from
    the initial state with the device steps.  The loss difference is formed node by node,
    sum (T+ - T-)(T+ + T- - 2 T*), so that the two large losses never cancel.  A gradient
    check of the reverse sweep (the time loop of Sec. II-A run backwards), not part of it."""
    import numpy as np
    tgt = dp.T_target.cpu().numpy()
    ids = dp.loss_ids.long()

    def final_T(kk, ww):
        dp.set_params(torch.as_tensor(kk, device=dp.dev), torch.as_tensor(ww, device=dp.dev))
        dp.reset()
        for _ in range(steps):
            dp.step(tol, precision)
        return dp.T[ids].cpu().numpy()

    a = final_T(k_e + h * dk, perf_e + h * dw)
    b = final_T(k_e - h * dk, perf_e - h * dw)
    return float(np.sum((a - b) * (a + b - 2.0 * tgt))) / (2.0 * h)
