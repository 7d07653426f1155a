"""torch.autograd interface to the Chambolle-Pock solve.

`cp_solve(problem, m0, V, n_iter, ...)` runs n_iter accelerated CP iterations
(eq. pasosChamPock, Section 5 schedule) from the initial point and returns the
final primal iterate y = (m, w) as a float64 CUDA tensor that is differentiable
with respect to m0 and V. The forward pass keeps a copy of the state every
`every` iterations; the backward pass is the library's reverse sweep
(mfg_cp_adjoint): it recomputes each segment from its checkpoint and runs one
solve with the symmetric reduced matrix (the same PCG) per reverse step.
The coupling and terminal cost are the problem's; `mbar` is the target density
of a terminal cost (problem.beta > 0), held fixed (not differentiated).
"""
from __future__ import annotations

import torch

from . import mfg


class _CPSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, m0, V, problem, n_iter, every, rtol, maxit, mbar):
        plan = mfg.mfg_plan(problem, V.detach().contiguous(), m0.detach().contiguous())
        if mbar is not None:
            mfg.mfg_set_target(plan, mbar.detach().contiguous())
        st = mfg.CPState(plan)
        mfg.mfg_cp_init(plan, st)
        ckpts = []
        done = 0
        while done < n_iter:
            ckpts.append(st.snapshot())
            k = min(every, n_iter - done)
            mfg.mfg_cp_solve(plan, st, k, rtol, maxit, stats=False)
            done += k
        if not ckpts:
            ckpts.append(st.snapshot())
        ctx.plan, ctx.ckpts = plan, ckpts
        ctx.args = (n_iter, every, rtol, maxit)
        return st.y.clone()

    @staticmethod
    def backward(ctx, gy):
        n_iter, every, rtol, maxit = ctx.args
        plan = ctx.plan
        g_m0 = torch.empty(plan.M, dtype=torch.float64, device=gy.device)
        g_V = torch.empty(plan.M, dtype=torch.float64, device=gy.device)
        mfg.mfg_cp_adjoint(plan, ctx.ckpts, every, n_iter, gy.contiguous(), rtol, maxit, g_m0,
                           g_V)
        ctx.ckpts = None
        return g_m0, g_V, None, None, None, None, None, None


def cp_solve(problem, m0, V, n_iter: int, rtol: float = 1e-10, maxit: int = 500,
             every: int = 10, mbar=None):
    """Final primal iterate after n_iter CP iterations; differentiable in m0, V."""
    return _CPSolve.apply(m0, V, problem, int(n_iter), int(every), float(rtol), int(maxit), mbar)


def terminal_m(problem, y):
    """m(., T): the last time slice of the density block of a primal vector."""
    M = problem.n[0] * (problem.n[1] if problem.d == 2 else 1)
    nt = problem.nt
    return y[(nt - 1) * M: nt * M]
