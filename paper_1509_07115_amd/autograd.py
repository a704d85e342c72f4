"""Differentiable multi-step propagation through the split-operator step.

One step (Sec. 4.1 with zero vector potential) is

    U_t = exp(-i s_t V tau/2) F^T T^T exp(-i K tau) T F exp(-i s_t V tau/2),

a product of unitary factors, so its adjoint U_t^H is the same sequence with
conjugated phases run in the opposite order (T^-1 = T^T, F^-1 = F^T: Sec. 2.4
and Appendix A).  ``propagate`` applies steps t = 0..n-1 with per-step potential
strengths s_t and returns psi_n; its backward pass is the adjoint method:

    lam_n = dL/dpsi_n (PyTorch convention, 2 dL/d conj(psi)),
    lam_t = U_t^H lam_{t+1},
    dL/ds_t = (tau/2) sum_i V_i Im(conj(lam_{t+1,i}) psi_{t+1,i} + conj(lam_{t,i}) psi_{t,i}),

and dL/dpsi_0 = lam_0.  The states psi_t are not kept: the forward pass stores
psi at every ``checkpoint_every``-th step, and the backward pass hands one
segment at a time to the library (``Plan.adjoint_segment``), which recomputes
the segment's states from its checkpoint and runs its adjoint steps and
reductions, from one captured graph per segment length when ``graph`` is set.
Every step runs in the library's kernels (``Plan.kinetic_step`` forward); this
module only orders the calls and holds tensors.
"""
from __future__ import annotations

import torch

__all__ = ["propagate"]


class _Propagate(torch.autograd.Function):
    @staticmethod
    def forward(ctx, psi0, s, plan, every, graph):
        nsteps = int(s.numel())
        s32 = s.detach().to(torch.float32).contiguous()
        psi = psi0.detach().clone(memory_format=torch.contiguous_format)
        ckpts = []
        for a in range(0, nsteps, every):
            n = min(every, nsteps - a)
            ckpts.append(psi.clone())
            plan.kinetic_step(psi, n, s32[a:a + n], graph=graph)
        ctx.plan, ctx.every, ctx.graph, ctx.s_dtype = plan, every, graph, s.dtype
        ctx.save_for_backward(s32, *ckpts)
        return psi

    @staticmethod
    def backward(ctx, grad_out):
        s32, *ckpts = ctx.saved_tensors
        plan, every, graph = ctx.plan, ctx.every, ctx.graph
        nsteps = int(s32.numel())
        lam = grad_out.detach().clone(memory_format=torch.contiguous_format)
        gs = torch.empty(nsteps, dtype=torch.float64, device=s32.device)
        # per segment, last first: recompute psi_a .. psi_{a+n} from the
        # checkpoint and run the n adjoint steps and strength gradients, all
        # in the library (one graph replay per segment when graph is set)
        for seg in range(len(ckpts) - 1, -1, -1):
            a = seg * every
            n = min(every, nsteps - a)
            plan.adjoint_segment(ckpts[seg], n, s32[a:a + n], lam, gs[a:a + n], graph=graph)
        g_s = gs.to(ctx.s_dtype) if ctx.needs_input_grad[1] else None
        g_psi = lam if ctx.needs_input_grad[0] else None
        return g_psi, g_s, None, None, None


def propagate(plan, psi0: torch.Tensor, s: torch.Tensor, checkpoint_every: int = 20,
              graph: bool = False) -> torch.Tensor:
    """psi_n = U_{n-1} ... U_0 psi0, differentiable in psi0 and in the strengths s.

    plan: a Plan with a potential set (``Plan.set_potential``); psi0: a device
    tensor in the plan's data layout and dtype; s: a real device tensor of n
    strengths; checkpoint_every: steps between stored states (memory: the
    len/checkpoint_every checkpoints, plus checkpoint_every + 3 state buffers
    that the plan holds for the backward pass); graph: capture each forward segment, and each backward segment, in a
    hipGraph.
    """
    if checkpoint_every < 1:
        raise ValueError("checkpoint_every must be >= 1")
    if s.dim() != 1 or s.numel() < 1:
        raise ValueError("s must be a 1-D tensor with at least one step")
    return _Propagate.apply(psi0, s, plan, int(checkpoint_every), bool(graph))
