"""Helpers shared by the GPU tests: build a GPU plan and the matching oracle
grid from one workload instance, and move arrays between NumPy and torch."""
import numpy as np

from oracle.grid import Grid


def grid_of(inst, l=None):
    d = inst.d
    return Grid(d=d, nx=inst.nx, ny=inst.ny, nt=inst.nt, bc=inst.bc, nu=inst.nu, T=inst.T,
                lo=tuple(inst.lo) + (0.0,) * (2 - d), hi=tuple(inst.hi) + (1.0,) * (2 - d),
                l=inst.l if l is None else l, gamma=inst.gamma)


def plan_of(inst, precision="fp64", l=None):
    import torch
    from paper_2507_01958_amd import mfg
    pb = mfg.make_problem(inst.d, inst.nx, inst.ny, inst.nt, inst.bc, inst.nu, inst.gamma,
                          l=inst.l if l is None else l, precision=precision, T=inst.T,
                          lo=inst.lo, hi=inst.hi)
    V = torch.from_numpy(inst.V).cuda()
    m0 = torch.from_numpy(inst.m0).cuda()
    return mfg.mfg_plan(pb, V, m0)


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def empty(n):
    import torch
    return torch.empty(n, dtype=torch.float64, device="cuda")


def say(msg):
    print(msg, flush=True)


def fp64_floor(g):
    """u * kappa(A) for the reduced matrix of eq. largeA: the scale of the
    forward error of any backward-stable float64 solve with it (u = 2^-53).
    lambda_max is bounded by the largest absolute row sum (Gershgorin) of the
    block rows C + I/dt^2 and -L/dt twice; lambda_min = lambda_1(l = 1)/dt^2,
    attained on spatially constant vectors."""
    from oracle import operators as ops
    from oracle import precond as pc
    S = ops.Spatial(g)
    rows = (np.asarray(abs(S.C).sum(axis=1)).ravel() + 1.0 / g.dt ** 2
            + 2.0 * np.asarray(abs(S.L).sum(axis=1)).ravel() / g.dt)
    lmin = pc.time_eigs(g.nt, 1)[0] / g.dt ** 2
    return 0.5 * np.finfo(float).eps * rows.max() / lmin
