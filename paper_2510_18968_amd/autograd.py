"""Differentiable rollout of the IMEX step: torch.autograd.Function wrappers
over the library's forward and adjoint entry points (no arithmetic here).

RMHDRollout runs n IMEX steps keeping (U, P) every `ckpt` steps (one
rmhd_steps call per segment); backward recomputes each segment forward from
its checkpoint with rmhd_step and applies rmhd_step_adjoint step by step in
reverse.  Prim2Con maps primitives to
conserved variables with rmhd_prim2con / rmhd_prim2con_adjoint.
"""
from __future__ import annotations

import torch


class Prim2Con(torch.autograd.Function):
    @staticmethod
    def forward(ctx, P, grid):
        ctx.grid = grid
        ctx.save_for_backward(P)
        return grid.prim2con(P.detach().contiguous())

    @staticmethod
    def backward(ctx, Ubar):
        (P,) = ctx.saved_tensors
        return ctx.grid.prim2con_adjoint(P.detach().contiguous(), Ubar.contiguous()), None


class RMHDRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, sigma, P0, grid, dt, nsteps, ckpt):
        U = U0.detach().clone()
        P = P0.detach().clone()
        sig = sigma.detach().contiguous()
        checkpoints = []
        # each segment in one rmhd_steps call (every final update runs the
        # next step's stage 1); backward recomputes the segment step by step
        for n0 in range(0, nsteps, ckpt):
            checkpoints.append((U.clone(), P.clone()))
            grid.steps(dt, sig, U, P, min(ckpt, nsteps - n0))
        if grid.failures():
            raise RuntimeError("recovery failures in the forward rollout")
        ctx.grid, ctx.dt, ctx.nsteps, ctx.ckpt = grid, dt, nsteps, ckpt
        ctx.checkpoints = checkpoints
        ctx.save_for_backward(sig)
        ctx.P_final = P
        return U

    @staticmethod
    def backward(ctx, Ubar):
        (sig,) = ctx.saved_tensors
        g, dt, nsteps, ckpt = ctx.grid, ctx.dt, ctx.nsteps, ctx.ckpt
        Ub = Ubar.detach().contiguous().clone()
        sbar = torch.zeros_like(sig)
        for s in reversed(range(len(ctx.checkpoints))):
            n0 = s * ckpt
            n1 = min(n0 + ckpt, nsteps)
            U, P = (t.clone() for t in ctx.checkpoints[s])
            states = []
            for _ in range(n0, n1):
                states.append((U.clone(), P.clone()))
                g.step(dt, sig, U, P)
            for Un, Pn in reversed(states):
                g.step_adjoint(dt, sig, Un, Pn, Ub, Ub, sbar)
        ctx.checkpoints = None
        # failed recoveries in the recomputed forward steps or singular
        # recovery Jacobians in the adjoint: the gradient is not trustworthy
        if g.failures():
            raise RuntimeError("recovery failures or singular recovery Jacobians in the backward rollout")
        return Ub, sbar, None, None, None, None, None


def rollout(U0, sigma, P0, grid, dt, nsteps, ckpt=20):
    return RMHDRollout.apply(U0, sigma, P0, grid, dt, nsteps, ckpt)


class SheetInversion:
    """The batch-of-current-sheets inverse problem: recover the per-problem
    conductivities from B^y at the final time.  Loss = sum over interior
    cells of (B^y(T) - B^y_target(T))^2, with the target evolved from the
    same initial data under a hidden per-problem sigma.  Parameters: the
    initial B^y field and log sigma per problem (the batch index is the y
    dimension of the grid)."""

    def __init__(self, w, grid, ckpt=20, steps=None):
        self.w, self.g, self.ckpt = w, grid, ckpt
        self.steps = w.steps if steps is None else steps
        dev = grid.device
        self.I = (slice(None),) + tuple(w.interior)
        self.P0 = torch.from_numpy(w.P.copy()).to(dev)
        self.target = self.final_By(self.P0[6], torch.tensor(w.extra["sigma_target"], device=dev).log()).detach()

    def sigma_field(self, log_sig):
        nprob = self.w.n[1]
        sig = torch.exp(log_sig).reshape(1, nprob, 1)
        return sig.expand(tuple(self.w.padded)).contiguous()

    def final_By(self, By0, log_sig):
        P0 = torch.cat([self.P0[:6], By0[None], self.P0[7:]], 0)
        U0 = Prim2Con.apply(P0, self.g)
        UT = rollout(U0, self.sigma_field(log_sig), P0.detach(), self.g, self.w.dt, self.steps, self.ckpt)
        return UT[6][self.I[1:]]

    def loss(self, By0, log_sig):
        return ((self.final_By(By0, log_sig) - self.target) ** 2).sum()
