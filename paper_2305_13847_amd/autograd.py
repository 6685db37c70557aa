"""torch.autograd wrappers over the library's adjoint calls.

The forward and backward passes call the C ABI only (dg_rhs / dg_rhs_vjp,
dg_saturation_split / dg_saturation_split_vjp, dg_rk_step / dg_rk_step_vjp);
torch holds the tensors and the checkpoints.
"""
from __future__ import annotations

import torch


class DGRhs(torch.autograd.Function):
    """dU/dt = rhs(U) with its hand-written vector-Jacobian product."""

    @staticmethod
    def forward(ctx, U, dg):
        ctx.dg = dg
        ctx.save_for_backward(U)
        return dg.rhs(U.contiguous())

    @staticmethod
    def backward(ctx, g):
        (U,) = ctx.saved_tensors
        return ctx.dg.rhs_vjp(U.contiguous(), g.contiguous()), None


class DGSplit(torch.autograd.Function):
    """(T, rho_v, rho_c) of the implicit-condensation split, differentiable in U."""

    @staticmethod
    def forward(ctx, U, dg):
        ctx.dg = dg
        ctx.save_for_backward(U)
        return dg.saturation_split(U.contiguous())

    @staticmethod
    def backward(ctx, Tb, rvb, rcb):
        (U,) = ctx.saved_tensors
        z = lambda x: None if x is None else x.contiguous()
        return ctx.dg.saturation_split_vjp(U.contiguous(), z(Tb), z(rvb), z(rcb)), None


class DGRollout(torch.autograd.Function):
    """nsteps SSP-RK steps with checkpoints every `every` steps.

    Forward keeps the state at every checkpoint; backward walks the segments
    in reverse, recomputes the states inside a segment and applies the
    one-step adjoint (which recomputes the stages) from the last step back.
    dt is fixed (it does not depend on the state).
    """

    @staticmethod
    def forward(ctx, U0, dg, dt, nsteps, every):
        ctx.dg, ctx.dt, ctx.nsteps, ctx.every = dg, dt, int(nsteps), int(every)
        U = U0.detach().clone().contiguous()
        ckpts = [U.clone()]
        done = 0
        while done < nsteps:
            k = min(every, nsteps - done)
            dg.rk_step(U, dt, k)
            done += k
            if done < nsteps:
                ckpts.append(U.clone())
        ctx.ckpts = ckpts
        return U

    @staticmethod
    def backward(ctx, g):
        dg, dt, every = ctx.dg, ctx.dt, ctx.every
        lam = g.contiguous().clone()
        out = torch.empty_like(lam)
        nseg = len(ctx.ckpts)
        for s in reversed(range(nseg)):
            start = s * every
            k = min(every, ctx.nsteps - start)
            states = [ctx.ckpts[s]]
            U = ctx.ckpts[s].clone()
            for _ in range(k - 1):
                dg.rk_step(U, dt, 1)
                states.append(U.clone())
            for Un in reversed(states):
                dg.rk_step_vjp(Un, lam, dt, out=out)
                lam, out = out, lam
        ctx.ckpts = None
        return lam, None, None, None, None


def rhs(U, dg):
    return DGRhs.apply(U, dg)


def split(U, dg):
    return DGSplit.apply(U, dg)


def rollout(U0, dg, dt, nsteps, every=20):
    return DGRollout.apply(U0, dg, dt, nsteps, every)
