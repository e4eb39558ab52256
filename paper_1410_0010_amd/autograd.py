"""torch.autograd wrappers of the solve with the hand-written reverse sweep.

Both functions run the forward solve through apm_solve and, on backward, the
reverse sweep apm_solve_adjoint, which reads the state the forward left in the
context: run backward before the next solve on the same context (otherwise the
library reports APM_ERR_STATE).  Gradients flow to the positions, masses and the
per-level packed gas tensors; owner grids are held fixed.
"""

from __future__ import annotations

from typing import List, Optional, Sequence

import torch

from .solver import Context


def _gas_list(ctx: Context, gas: Sequence[Optional[torch.Tensor]]):
    gas = list(gas)
    if len(gas) != ctx.plan.nlevels:
        raise ValueError(f"expected {ctx.plan.nlevels} gas entries (None allowed), got {len(gas)}")
    return gas if any(g is not None for g in gas) else None


class APMSolve(torch.autograd.Function):
    """(x, y, z, m, *gas) -> (ax, ay, az, pot) per particle."""

    @staticmethod
    def forward(fctx, ctx: Context, x, y, z, m, *gas):
        g = _gas_list(ctx, gas) if gas else None
        ax, ay, az, pot = ctx.solve(x, y, z, m, g)
        fctx.apm = ctx
        fctx.gas = g
        fctx.save_for_backward(x, y, z, m, pot)
        return ax, ay, az, pot

    @staticmethod
    def backward(fctx, gax, gay, gaz, gpot):
        x, y, z, m, pot = fctx.saved_tensors
        ctx, g = fctx.apm, fctx.gas
        c = lambda t: None if t is None else t.contiguous()
        xb, yb, zb, mb, gb = ctx.solve_adjoint(x, y, z, m, g, pot, (c(gax), c(gay), c(gaz)),
                                               c(gpot), 0.0, want_gas=g is not None)
        gas_grads = gb if gb is not None else [None] * (len(fctx.needs_input_grad) - 5)
        return (None, xb, yb, zb, mb, *gas_grads)


class APMEnergy(torch.autograd.Function):
    """(x, y, z, m, *gas) -> W, the potential energy of the solve (FP64 scalar)."""

    @staticmethod
    def forward(fctx, ctx: Context, x, y, z, m, *gas):
        g = _gas_list(ctx, gas) if gas else None
        ax, ay, az, pot = ctx.solve(x, y, z, m, g)
        tot = ctx.solve_totals(m, ax, ay, az, pot, gas=g)
        fctx.apm = ctx
        fctx.gas = g
        fctx.save_for_backward(x, y, z, m, pot)
        return torch.tensor(tot[ctx.plan.nlevels], dtype=torch.float64, device=x.device)

    @staticmethod
    def backward(fctx, gw):
        x, y, z, m, pot = fctx.saved_tensors
        ctx, g = fctx.apm, fctx.gas
        xb, yb, zb, mb, gb = ctx.solve_adjoint(x, y, z, m, g, pot, None, None, float(gw.item()),
                                               want_gas=g is not None)
        gas_grads = gb if gb is not None else [None] * (len(fctx.needs_input_grad) - 5)
        return (None, xb, yb, zb, mb, *gas_grads)


def solve(ctx: Context, x, y, z, m, gas: Optional[List[Optional[torch.Tensor]]] = None):
    """Differentiable forward solve: (ax, ay, az, pot)."""
    return APMSolve.apply(ctx, x, y, z, m, *(gas or []))


def potential_energy(ctx: Context, x, y, z, m, gas: Optional[List[Optional[torch.Tensor]]] = None):
    """Differentiable potential energy W (particles + gas)."""
    return APMEnergy.apply(ctx, x, y, z, m, *(gas or []))
