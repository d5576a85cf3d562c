"""torch.autograd wrapper of the DP value and its hand-written adjoint.

``EcoDPValue.apply(theta, inst)`` returns V_0(x0; theta) (FP64 scalar) for
theta = (M, CdA, Crr, w_t, w_soc); its backward runs ``dp_adjoint`` on the GPU
(the occupancy sweep with the argmin policy held fixed) and returns
grad_out * dV_0/dtheta.
"""
from __future__ import annotations

import torch

from .api import Plan


class EcoDPValue(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta: torch.Tensor, inst: dict, device: int = 0):
        x = dict(inst)
        x["theta"] = [float(v) for v in theta.detach().to("cpu", torch.float64).tolist()]
        plan = Plan([x], store_all=True, device=device)
        V0, _ = plan.solve()
        ctx.plan = plan
        return V0[0].to(torch.float64).to(theta.device)

    @staticmethod
    def backward(ctx, grad_out):
        g = ctx.plan.adjoint()[0].to(grad_out.device)
        return grad_out * g, None, None
