"""torch.autograd wrapper of the propagation: forward = pc_propagate_batched keeping only
the segment-boundary states (checkpoints), backward = pc_adjoint (reverse sweep that
re-solves each segment from its checkpoint).  Argument marshalling only."""
from __future__ import annotations

import torch

from . import pcprop


class PCPropagate(torch.autograd.Function):
    """states (and optionally node states) of ``ics`` propagated through ``groups``."""

    @staticmethod
    def forward(ctx, ics, pc, groups, model, opts, return_nodes, adj_tol):
        r = pc.propagate_batched(ics.detach().contiguous(), groups, model, want_bounds=True,
                                 want_nodes=return_nodes, raise_on_status=True, **opts)
        ctx.save_for_backward(r["bounds"])
        ctx.pc, ctx.groups, ctx.model, ctx.opts, ctx.adj_tol = pc, groups, model, opts, adj_tol
        if return_nodes:
            return r["states"], r["nodes"]
        return r["states"]

    @staticmethod
    def backward(ctx, grad_states, grad_nodes=None):
        (bounds,) = ctx.saved_tensors
        if grad_states is None:
            grad_states = torch.zeros((bounds.shape[0], 6), dtype=bounds.dtype, device=bounds.device)
        gn = grad_nodes.contiguous() if grad_nodes is not None else None
        grad, _, _ = ctx.pc.adjoint(bounds, grad_states.contiguous(), ctx.groups, ctx.model, gbar_nodes=gn,
                                    adj_tol=ctx.adj_tol, raise_on_status=True, **ctx.opts)
        return grad, None, None, None, None, None, None


def propagate(ics, groups, model=None, *, return_nodes=False, adj_tol=1e-12, pc=None, **opts):
    """Differentiable propagation: returns states [n, 6] (and node states [n, S, N, 6])."""
    pc = pc or pcprop.context(ics.device.index)
    return PCPropagate.apply(ics, pc, groups, model or pcprop.Model(), opts, return_nodes, adj_tol)
