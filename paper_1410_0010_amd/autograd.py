"""torch.autograd wrappers of the solve with the hand-written reverse sweep.

Both functions run the forward solve through apm_solve and, on backward, the
reverse sweep apm_solve_adjoint, which reads the state the forward left in the
context: run backward before the next solve on the same context.  A backward after
a later solve on the context raises (the context counts its solves; the library's
own check on the particle and gas pointers reports APM_ERR_STATE as well).  The gas
tensors are saved for backward, so torch reports their in-place modification.
Gradients flow to the positions, masses and the per-level packed gas tensors; owner
grids are held fixed.
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


def _save(fctx, ctx: Context, g, x, y, z, m, pot):
    fctx.apm = ctx
    fctx.gen = ctx.solve_count
    fctx.nlev = ctx.plan.nlevels
    fctx.has_gas = [t is not None for t in g] if g is not None else None
    fctx.save_for_backward(x, y, z, m, pot, *[t for t in (g or []) if t is not None])


def _restore(fctx):
    ctx = fctx.apm
    if ctx.solve_count != fctx.gen:
        raise RuntimeError("APM backward: another solve ran on this context after the forward "
                           "of this graph; its reverse sweep needs the forward's state")
    x, y, z, m, pot, *gs = fctx.saved_tensors
    g = None
    if fctx.has_gas is not None:
        it = iter(gs)
        g = [next(it) if h else None for h in fctx.has_gas]
    return ctx, g, x, y, z, m, pot


class APMSolve(torch.autograd.Function):
    """(x, y, z, m, *gas) -> (ax, ay, az, pot) per particle."""

    @staticmethod
    def forward(fctx, ctx: Context, x, y, z, m, *gas):
        g = _gas_list(ctx, gas) if gas else None
        ax, ay, az, pot = ctx.solve(x, y, z, m, g)
        _save(fctx, ctx, g, x, y, z, m, pot)
        return ax, ay, az, pot

    @staticmethod
    def backward(fctx, gax, gay, gaz, gpot):
        ctx, g, x, y, z, m, pot = _restore(fctx)
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
        _save(fctx, ctx, g, x, y, z, m, pot)
        return torch.tensor(tot[ctx.plan.nlevels], dtype=torch.float64, device=x.device)

    @staticmethod
    def backward(fctx, gw):
        ctx, g, x, y, z, m, pot = _restore(fctx)
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
