"""High-level entry points over the C ABI (argument marshalling only)."""
from __future__ import annotations

import torch

from . import native


def params_tensor(batch, device="cuda") -> torch.Tensor:
    """The batch's float64 parameter array as a device tensor."""
    return torch.as_tensor(batch.params, dtype=torch.float64).to(device).contiguous()


def integrate(batch, precision: str = "fp64", params=None, with_bound: bool = False, plan=None,
              block_dims: int = 0):
    """Smolyak values (2.6) of every integrand of ``batch`` on the GPU.

    Returns (values, bounds or None) as float64 device tensors in problem
    order.  ``params`` overrides the batch's parameters (a device tensor).
    ``block_dims`` > 0 selects the block (tensor-product) variant of the
    rule with blocks of that many coordinates (Algorithm 3.3, step m).
    """
    if params is None:
        params = params_tensor(batch)
    own = plan is None
    plan = plan or native.Plan(batch.problems, precision, block_dims=block_dims)
    try:
        out = torch.empty(len(batch), dtype=torch.float64, device=params.device)
        bound = torch.empty_like(out) if with_bound else None
        plan.execute(params, out, bound)
        return out, bound
    finally:
        if own:
            plan.close()


class SGIntegral(torch.autograd.Function):
    """Q(params) for a fixed plan, with the library's reverse sweep as backward."""

    @staticmethod
    def forward(ctx, params, plan):
        ctx.plan = plan
        ctx.save_for_backward(params)
        return plan.execute(params.contiguous())

    @staticmethod
    def backward(ctx, grad_out):
        (params,) = ctx.saved_tensors
        g = ctx.plan.execute_grad(params.contiguous(), grad_out.contiguous().to(torch.float64))
        return g, None
