"""torch.autograd wrapper of the propagation: forward = pc_propagate_batched keeping the
segment-boundary states (checkpoints) and, when asked, the converged node states;
backward = pc_adjoint (reverse sweep that re-solves each segment from its checkpoint, or
reads its node states when they were kept).  Argument marshalling only."""
from __future__ import annotations

import torch

from . import pcprop


class PCPropagate(torch.autograd.Function):
    """states (and optionally node states) of ``ics`` propagated through ``groups``."""

    @staticmethod
    def forward(ctx, ics, pc, groups, model, opts, return_nodes, adj_tol, store_nodes):
        r = pc.propagate_batched(ics.detach().contiguous(), groups, model, want_bounds=True,
                                 want_nodes=return_nodes or store_nodes, raise_on_status=True, **opts)
        ctx.store_nodes = store_nodes
        if store_nodes:
            ctx.save_for_backward(r["bounds"], r["nodes"])
        else:
            ctx.save_for_backward(r["bounds"])
        ctx.pc, ctx.groups, ctx.model, ctx.opts, ctx.adj_tol = pc, groups, model, opts, adj_tol
        if return_nodes:
            return r["states"], r["nodes"]
        return r["states"]

    @staticmethod
    def backward(ctx, grad_states, grad_nodes=None):
        saved = ctx.saved_tensors
        bounds = saved[0]
        fwd_nodes = saved[1] if ctx.store_nodes else None
        if grad_states is None:
            grad_states = torch.zeros((bounds.shape[0], 6), dtype=bounds.dtype, device=bounds.device)
        gn = grad_nodes.contiguous() if grad_nodes is not None else None
        grad, _, _ = ctx.pc.adjoint(bounds, grad_states.contiguous(), ctx.groups, ctx.model, gbar_nodes=gn,
                                    adj_tol=ctx.adj_tol, raise_on_status=True, fwd_nodes=fwd_nodes, **ctx.opts)
        return grad, None, None, None, None, None, None, None


def propagate(ics, groups, model=None, *, return_nodes=False, adj_tol=1e-12, store_nodes=False, pc=None,
              **opts):
    """Differentiable propagation: returns states [n, 6] (and node states [n, S, N, 6]).

    ``store_nodes``: keep the converged node states for the backward pass (48 bytes per IC,
    node and segment) instead of only the segment checkpoints, so that it reads them
    rather than re-solving every segment."""
    pc = pc or pcprop.context(ics.device.index)
    return PCPropagate.apply(ics, pc, groups, model or pcprop.Model(), opts, return_nodes, adj_tol, store_nodes)
