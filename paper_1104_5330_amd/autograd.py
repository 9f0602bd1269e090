"""torch.autograd bindings of the RK4 transport step and of the outgoing-flux map.

TransportRK4.apply(grid, F0, kappa, sigma, eta, dt, n_steps, checkpoint_every,
keep_stages) runs n_steps RK4 steps (sp6_step) and keeps the state every
checkpoint_every steps; the backward pass recomputes each segment from its
checkpoint and walks it in reverse with the discrete adjoint, which also
accumulates the gradients of kappa, eta and sigma.  With keep_stages the
recomputation keeps every step's stage inputs (sp6_step_stages: four states per
step of the segment in memory) and the adjoint reads them
(sp6_adjoint_step_stages); without, it keeps one state per step
(sp6_step) and the adjoint recomputes the stages (sp6_adjoint_step).  The
results are the same.  OutgoingFlux.apply(grid, F)
is the flux map at r_out with its transpose as backward.  Both only marshal
tensors; every arithmetic step runs in the HIP library.
"""

import torch


class TransportRK4(torch.autograd.Function):
    @staticmethod
    def forward(ctx, grid, F0, kappa, sigma, eta, dt, n_steps, checkpoint_every, keep_stages=True):
        K = max(1, int(checkpoint_every))
        grid.set_coefficients(kappa.contiguous(), sigma.contiguous(), eta.contiguous())
        F = F0.detach().clone().contiguous()
        ckpts = [F.clone()]
        done = 0
        while done < n_steps:
            n = min(K, n_steps - done)
            grid.step(F, dt, n)
            done += n
            if done < n_steps:
                ckpts.append(F.clone())
        ctx.grid, ctx.dt, ctx.n_steps, ctx.K, ctx.keep = grid, dt, n_steps, K, bool(keep_stages)
        ctx.ckpts = ckpts
        ctx.save_for_backward(kappa, sigma, eta)
        return F

    @staticmethod
    def backward(ctx, gF):
        grid, dt, n_steps, K = ctx.grid, ctx.dt, ctx.n_steps, ctx.K
        kappa, sigma, eta = ctx.saved_tensors
        grid.set_coefficients(kappa.contiguous(), sigma.contiguous(), eta.contiguous())
        lam = gF.detach().clone().contiguous()
        gk = torch.zeros_like(kappa)
        ge = torch.zeros_like(eta)
        gs = torch.zeros_like(sigma)
        for seg in reversed(range(len(ctx.ckpts))):
            n = min(K, n_steps - seg * K)
            states = [ctx.ckpts[seg]]
            if ctx.keep:
                stages = []
                for i in range(n):
                    Ys = torch.empty((3,) + tuple(states[-1].shape), dtype=states[-1].dtype,
                                     device=states[-1].device)
                    s = states[-1].clone()
                    grid.step_stages(s, dt, Ys)
                    stages.append(Ys)
                    if i < n - 1:
                        states.append(s)
                for s, Ys in zip(reversed(states), reversed(stages)):
                    grid.adjoint_step_stages(s, Ys, dt, lam, gk, ge, gs)
                stages.clear()
            else:
                for _ in range(n - 1):
                    s = states[-1].clone()
                    grid.step(s, dt, 1)
                    states.append(s)
                for s in reversed(states):
                    grid.adjoint_step(s, dt, lam, gk, ge, gs)
            states.clear()
        ctx.ckpts = None
        return None, lam, gk, gs, ge, None, None, None, None


class OutgoingFlux(torch.autograd.Function):
    @staticmethod
    def forward(ctx, grid, F):
        ctx.grid = grid
        return grid.outgoing_flux(F.contiguous())

    @staticmethod
    def backward(ctx, gj):
        return None, ctx.grid.outgoing_flux_T(gj.contiguous())


def transport(grid, F0, kappa, sigma, eta, dt, n_steps, checkpoint_every=20, keep_stages=True):
    return TransportRK4.apply(grid, F0, kappa, sigma, eta, dt, n_steps, checkpoint_every, keep_stages)


def outgoing_flux(grid, F):
    return OutgoingFlux.apply(grid, F)
