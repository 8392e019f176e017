"""Differentiable mapmaking: a torch.autograd.Function around the library's solve.

Forward: the cooled messenger solve (Section 3.1 schedule) of eqn. (mapmaking) for the
current noise parameters.  Backward: implicit differentiation of the solved map
m = A^-1 P^T N^-1 d, A = P^T N^-1 P.  For g = dL/dm the adjoint map z = A^-1 g comes
from re-running a solve of the same symmetric system; then

    dL/dd       = N^-1 P z                                   (mm_tod_apply)
    dL/dtheta_c = -(1/n_c) sum_k omega_k Re(conj(zhat_k) rhat_k) dN_k/dtheta_c / N_k^2
                                                             (mm_noise_grad)

with r = d - P m and theta = (sigma, fknee, alpha) per chunk.  Only the solved map and the
data are kept for the backward pass (the gradient needs no intermediate iterate).

The adjoint solve is preconditioned CG on A with the map-space right-hand side g (the
default), or the cooled messenger solve on the lifted data N T^-1 P W^-1 g
(adjoint="messenger"); the lift multiplies by N/tau, whose range reaches N(f_1)/sigma^2
(~1e12 for steep 1/f noise), so the messenger route is only accurate for mild noise.
Every numeric step runs in libmm; this module only sequences the calls.
"""

from __future__ import annotations

from typing import Optional, Sequence

import numpy as np
import torch

from . import mm


def _noise_changed(plan, sigma, fknee, alpha, tau) -> bool:
    cur = getattr(plan, "_noise", None)
    new = (tuple(sigma), tuple(fknee), tuple(alpha), None if tau is None else tuple(tau))
    if cur != new:
        plan._noise = new
        return True
    return False


class MessengerSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, d: torch.Tensor, sigma: torch.Tensor, fknee: torch.Tensor, alpha: torch.Tensor,
                plan: mm.Plan, lambdas: Sequence[float], iters: Sequence[int], adjoint: str = "cg",
                adjoint_iters: int = 500, adjoint_rtol: float = 1e-10, tau=None):
        s = sigma.detach().double().cpu().numpy()
        f = fknee.detach().double().cpu().numpy()
        a = alpha.detach().double().cpu().numpy()
        # the messenger variance: the given one, else whatever the plan was last given (its
        # default sigma^2 when it never was)
        t = np.asarray(tau, dtype=np.float64).reshape(-1) if tau is not None else plan.tau
        if _noise_changed(plan, s, f, a, t):
            mm.mm_plan_set_noise(plan, s, f, a, t)
        m = torch.zeros(plan.map_shape, dtype=torch.float64, device=d.device)
        dd = d.detach().to(plan.tod_dtype).contiguous()
        mm.mm_solve(plan, dd, lambdas, iters, m)
        ctx.plan = plan
        ctx.noise = (s, f, a, t)
        ctx.sched = (list(lambdas), list(iters))
        ctx.adjoint = (adjoint, adjoint_iters, adjoint_rtol)
        ctx.d_dtype = d.dtype
        ctx.theta = (sigma.device, sigma.dtype)
        ctx.save_for_backward(dd, m)
        return m

    @staticmethod
    def backward(ctx, gm: torch.Tensor):
        dd, m = ctx.saved_tensors
        plan = ctx.plan
        # another forward may have set other noise parameters on the plan since this one ran
        if _noise_changed(plan, *ctx.noise):
            mm.mm_plan_set_noise(plan, *ctx.noise)
        g = gm.detach().double().contiguous()
        z = torch.zeros_like(m)
        kind, maxit, rtol = ctx.adjoint
        if kind == "messenger":
            dg = torch.empty_like(dd)
            mm.mm_lift_rhs(plan, g, dg)
            mm.mm_solve(plan, dg, ctx.sched[0], ctx.sched[1], z)
        else:
            mm.mm_cg_solve(plan, z, maxit, rhs_map=g, rtol=rtol)
        grad_d = grad_s = grad_f = grad_a = None
        if ctx.needs_input_grad[0]:
            out = torch.empty_like(dd)
            mm.mm_tod_apply(plan, 0, z, out)
            grad_d = out.to(ctx.d_dtype)
        if any(ctx.needs_input_grad[1:4]):
            gr = torch.empty((plan.nchunk, 3), dtype=torch.float64, device=m.device)
            mm.mm_noise_grad(plan, dd, m, z, gr)
            gr = gr.to(device=ctx.theta[0], dtype=ctx.theta[1])
            grad_s, grad_f, grad_a = gr[:, 0].contiguous(), gr[:, 1].contiguous(), gr[:, 2].contiguous()
        return grad_d, grad_s, grad_f, grad_a, None, None, None, None, None, None, None


def messenger_solve(d, sigma, fknee, alpha, plan, lambdas, iters, adjoint: str = "cg", adjoint_iters: int = 500,
                    adjoint_rtol: float = 1e-10, tau=None):
    """Differentiable solved map (see MessengerSolve).  ``tau`` (per chunk, not differentiated)
    sets the messenger variance; by default the plan keeps the one it was built or last set with."""
    return MessengerSolve.apply(d, sigma, fknee, alpha, plan, lambdas, iters, adjoint, adjoint_iters, adjoint_rtol,
                                tau)
