"""torch.autograd.Function for the registration objective J(v).

Forward runs the library's state solve and objective; backward returns the
hand-written adjoint gradient (Section "Optimality Conditions": adjoint
equation e:first-order-adjoint and reduced gradient e:first-order-control,
eliminated form e:eliminated-control). The library's gradient is the L2-Riesz
representative g with dJ[w] = h_d sum(g w); autograd works with the Euclidean
(l2) gradient dJ/dv = h_d g, so backward multiplies by h_d.
"""
from __future__ import annotations

import torch


class RegistrationObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, v: torch.Tensor, problem) -> torch.Tensor:
        vc = v.detach().contiguous()
        J, Jd, Jr, g = problem.objective_gradient(vc)
        ctx.save_for_backward(g)
        ctx.hd = problem.hd
        return torch.tensor(J, dtype=torch.float64, device=v.device)

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        (g,) = ctx.saved_tensors
        return (grad_out.to(g.dtype) * ctx.hd) * g, None


def objective(v: torch.Tensor, problem) -> torch.Tensor:
    """J(v) as a differentiable scalar (FP64) whose gradient comes from the adjoint solve."""
    return RegistrationObjective.apply(v, problem)
