"""torch.autograd entry to the parameter derivatives of the QTT step.

``final_statistic(omega, k_react, workload, n_steps)`` returns, as a 0-d
torch tensor, a linear statistic of the PDF after n_steps explicit RK steps
of the workload with Omega_mix = omega and C_r = k_react.  Its backward
returns dJ/domega and dJ/dk_react, which the forward pass computes alongside
the state with tt_step_tangent (forward-mode tangents of the discrete step,
carried through every stage and rounding on the GPU).  Only the two scalar
parameters are differentiable.
"""
from __future__ import annotations

import torch

from . import Context, statistic_and_gradient


class _FinalStatistic(torch.autograd.Function):
    @staticmethod
    def forward(ctx, omega, k_react, workload, n_steps, statistic, dtype, qctx):
        w = workload.replace(omega=float(omega), k_react=float(k_react))
        J, g = statistic_and_gradient(qctx, w, n_steps, statistic, dtype)
        ctx.save_for_backward(torch.tensor([g["omega"], g["k_react"]], dtype=torch.float64))
        return torch.tensor(J, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gJ):
        (g,) = ctx.saved_tensors
        return gJ * g[0], gJ * g[1], None, None, None, None, None


def final_statistic(omega, k_react, workload, n_steps, statistic="product", dtype="f64", qctx=None):
    """J(omega, k_react) = statistic(f(T)); differentiable in omega and k_react."""
    qctx = qctx if qctx is not None else Context(0)
    om = torch.as_tensor(omega, dtype=torch.float64)
    kr = torch.as_tensor(k_react, dtype=torch.float64)
    return _FinalStatistic.apply(om, kr, workload, n_steps, statistic, dtype, qctx)
