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


_U64 = 2.0 ** -53


def box_to_unit(family: str, params, d: int, lo, hi):
    """Reparameterise an integrand on the box [lo, hi]^d (lo, hi scalars or
    length-d arrays, lo < hi) onto the unit cube of the rule (2.6):
    x = lo + L t, L = hi - lo.  Returns (unit_params, factor, factor_rel_err)
    with  integral over the box of f = factor * integral over [0,1]^d of the
    mapped integrand, and factor's relative rounding error bound.  Each
    family keeps its form: exp-sum c' = c L (factor exp(sum c lo));
    oscillatory a' = a L, w' = w + sum a lo / (2 pi); product-peak b' = b L,
    u' = (u - lo) / L (factor prod L^-2); corner-peak a' = a L / S0 with
    S0 = 1 + sum a lo > 0 (factor S0^-(d+1)); gaussian c' = c L^2,
    u' = (u - lo) / L; the oscillatory quadratics a' = a L^2,
    u' = (u - lo) / L and, for the linear term, c' = c L,
    w' = w + sum c lo / (2 pi).  Every factor also carries the box volume
    prod L.  The mapped parameters are rounded once each (in FP64): the rule
    then integrates that rounded integrand."""
    import math

    import numpy as np
    p = np.asarray(params, dtype=np.float64)
    lo = np.broadcast_to(np.asarray(lo, dtype=np.float64), (d,)).copy()
    hi = np.broadcast_to(np.asarray(hi, dtype=np.float64), (d,)).copy()
    L = hi - lo
    if not np.all(L > 0):
        raise ValueError("box_to_unit: every hi must exceed its lo")
    vol = float(np.prod(L))
    rel = (d + 1) * _U64          # the volume's products
    two_pi = 2.0 * math.pi
    if family == "exp_sum":
        c = p[:d]
        s0 = float(np.sum(c * lo))
        return c * L, vol * math.exp(s0), rel + (d + 1) * _U64 * float(np.sum(np.abs(c * lo))) + 2 * _U64
    if family == "oscillatory":
        w, a = p[0], p[1:1 + d]
        w2 = math.fmod(w + float(np.sum(a * lo)) / two_pi, 1.0)
        return np.concatenate([[w2], a * L]), vol, rel
    if family == "product_peak":
        b, u = p[:d], p[d:2 * d]
        return np.concatenate([b * L, (u - lo) / L]), vol * float(np.prod(L ** -2.0)), rel + (3 * d + 2) * _U64
    if family == "corner_peak":
        a = p[:d]
        s0 = 1.0 + float(np.sum(a * lo))
        if not s0 > 0:
            raise ValueError("box_to_unit: corner-peak needs 1 + sum a lo > 0")
        s0_rel = (d + 1) * _U64 * (1.0 + float(np.sum(np.abs(a * lo)))) / s0
        return a * L / s0, vol * s0 ** (-(d + 1)), rel + (d + 1) * s0_rel + 4 * _U64
    if family == "gaussian":
        c, u = p[:d], p[d:2 * d]
        return np.concatenate([c * L * L, (u - lo) / L]), vol, rel
    if family in ("oscillatory_quadratic", "oscillatory_quadratic_linear"):
        w, a, u = p[0], p[1:1 + d], p[1 + d:1 + 2 * d]
        out = [a * L * L, (u - lo) / L]
        if family == "oscillatory_quadratic_linear":
            c = p[1 + 2 * d:1 + 3 * d]
            w = w + float(np.sum(c * lo)) / two_pi
            out.append(c * L)
        return np.concatenate([[math.fmod(w, 1.0)]] + out), vol, rel
    raise ValueError(f"unknown family {family!r}")


def integrate_one(family: str, params, d: int, q: int, rule: str, precision: str = "fp64", box=None,
                  with_bound: bool = False):
    """One integrand on the plan-free path (sg_integrate): the Smolyak value
    (2.6) of f over [0,1]^d, or over the box [lo, hi]^d given as box=(lo, hi)
    (box_to_unit, on the host).  Returns the value (and, with with_bound,
    the stated rounding bound: the library's bound times |factor| plus the
    factor's own rounding) as Python floats."""
    import numpy as np
    from .workloads import Problem
    factor, frel = 1.0, 0.0
    prm = np.asarray(params, dtype=np.float64)
    if box is not None:
        prm, factor, frel = box_to_unit(family, prm, d, box[0], box[1])
    pr = torch.as_tensor(prm, dtype=torch.float64).cuda()
    out = torch.empty(1, dtype=torch.float64, device=pr.device)
    bound = torch.empty_like(out) if with_bound else None
    native.integrate_one(Problem(d, q, rule, family, 0), pr, precision, out=out, bound=bound)
    v = out.item()
    val = factor * v
    if not with_bound:
        return val
    return val, abs(factor) * bound.item() * (1 + 2 * _U64) + (frel + 2 * _U64) * abs(val)


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
