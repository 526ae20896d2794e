"""Differentiable time loop: soma voltage traces of an implicit-Euler
simulation as a function of the edge conductances a, the capacitive terms c
and the injected currents I, with a hand-written adjoint.

Forward (paper §1, the current evaluated at the old step):
    A V^k = c V^{k-1} + I,  V^0 = 0,  A = diag(c) + L(a),  k = 1 .. steps,
    traces[k-1, cell] = V^k at the cell's root.
Backward, given G[k-1, cell] = dLoss/dtraces[k-1, cell]; A is symmetric, so
each adjoint step is one more solve with the same matrix:
    lambda^{steps+1} = 0;  for k = steps .. 1:
        A lambda^k = c lambda^{k+1} + G[k-1] at the roots
        dL/dI   += lambda^k
        dL/dc_i += lambda^k_i (V^{k-1}_i - V^k_i)
        dL/da_i += -(lambda^k_i - lambda^k_p)(V^k_i - V^k_p),  p = parent(i)
States are checkpointed every ``checkpoint_every`` steps and recomputed one
segment at a time during the backward pass; the kernels are deterministic,
so the recomputed states equal the forward ones bit for bit.

All arithmetic runs in the library's kernels (hines_assemble, hines_timestep,
hines_gather_roots, hines_adjoint_rhs, hines_solve, hines_adjoint_accumulate);
torch provides the device buffers.
"""
from __future__ import annotations

import torch


class _SomaTraces(torch.autograd.Function):
    @staticmethod
    def forward(ctx, a, c, I, plan, steps, checkpoint_every):
        a = a.contiguous()
        c = c.contiguous()
        I = I.contiguous()
        diag, upper = plan.assemble(a, c)
        V = torch.zeros_like(c)
        traces = torch.empty(steps, plan.ncells, dtype=torch.float64, device=c.device)
        ckpts = [V.clone()]
        for k in range(1, steps + 1):
            plan.timestep(diag, upper, c, V, V, i_inj=I, step=k - 1)
            plan.gather_roots(V, out=traces[k - 1])
            if k % checkpoint_every == 0 and k < steps:
                ckpts.append(V.clone())
        ctx.plan = plan
        ctx.steps = steps
        ctx.every = checkpoint_every
        ctx.save_for_backward(c, I, diag, upper, *ckpts)
        return traces

    @staticmethod
    def backward(ctx, G):
        plan, steps, every = ctx.plan, ctx.steps, ctx.every
        c, I, diag, upper, *ckpts = ctx.saved_tensors
        G = G.contiguous()
        ga = torch.zeros_like(c)
        gc = torch.zeros_like(c)
        gi = torch.zeros_like(c)
        lam_next = None
        nseg = (steps + every - 1) // every
        for s in range(nseg - 1, -1, -1):
            k0 = s * every
            k1 = min(k0 + every, steps)
            states = [ckpts[s]]
            V = ckpts[s].clone()
            for k in range(k0 + 1, k1 + 1):
                plan.timestep(diag, upper, c, V, V, i_inj=I, step=k - 1)
                states.append(V.clone())
            for k in range(k1, k0, -1):
                mu = plan.adjoint_rhs(c, lam_next, G[k - 1])
                lam = plan.solve(diag, upper, mu)
                plan.adjoint_accumulate(lam, states[k - k0], states[k - 1 - k0], ga, gc, gi)
                lam_next = lam
        return ga, gc, gi, None, None, None


def soma_traces(plan, a, c, I, steps: int, checkpoint_every: int = 10):
    """Soma voltages [steps, ncells] of the simulation, differentiable w.r.t.
    a (edge conductance stored at the child; roots ignored), c and I."""
    return _SomaTraces.apply(a, c, I, plan, int(steps), int(checkpoint_every))
