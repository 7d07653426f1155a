"""Accelerated Chambolle-Pock iteration on (VMFG_h) (Section 3, Section 5).

With phi = B-hat + F and psi the indicator of {G(m, w) = 0}, one iteration
(eq. pasosChamPock, written here with xi for the dual variable) is
    xi_{l+1}   = prox_{sigma psi*}(xi_l + sigma ybar_l)
               = Cr^T (Cr Cr^T)^{-1} (Cr (xi_l + sigma ybar_l) - sigma dr)   (eq. CC*)
    y_{l+1}    = prox_{tau phi}(y_l - tau xi_{l+1})
    ybar_{l+1} = y_{l+1} + theta (y_{l+1} - y_l)
with the step-size schedule of Section 5: tau_0 = sigma_0 = 1 in the first
iteration; after iteration l, theta = (1 + 2 gamma tau_l)^{-1/2},
tau_{l+1} = theta tau_l, sigma_{l+1} = sigma_l / theta, and the extrapolation
uses that theta (the ordering of Chambolle and Pock's accelerated scheme).
Initial point: xi_0 = 0, y_0 = ybar_0 = (m_0 at every time slice, w = 0).
The cost phi is b-hat + F with the coupling and terminal cost given by a
prox.Coupling (default f = m + V, g = 0).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse.linalg as spla

from . import cg as cgmod
from . import operators as ops
from .grid import Grid
from .precond import apply_Pinv_fast
from .prox import LINEAR, Coupling, prox_primal


@dataclasses.dataclass
class CPState:
    xi: np.ndarray
    y: np.ndarray
    ybar: np.ndarray
    sigma: float = 1.0
    tau: float = 1.0
    theta: float = 1.0
    it: int = 0

    def copy(self):
        return CPState(self.xi.copy(), self.y.copy(), self.ybar.copy(), self.sigma,
                       self.tau, self.theta, self.it)


def cp_init(g: Grid, m0: np.ndarray) -> CPState:
    nb = 1 + g.ncomp
    y = np.zeros(nb * g.n)
    y[: g.n] = np.tile(m0, g.nt)
    return CPState(np.zeros(nb * g.n), y, y.copy())


class Projector:
    """Solves A u = b for the projection with the chosen method:
    'cg' (plain CG), 'pcg' (CG preconditioned by Algorithms 1+2, computed
    with a dense V and scipy.fft), 'direct' (sparse LU of the assembled
    matrix; small grids)."""

    def __init__(self, g: Grid, S: ops.Spatial, method: str, rtol: float, maxit: int):
        self.g, self.S, self.method, self.rtol, self.maxit = g, S, method, rtol, maxit
        self._lu = None
        if method == "direct":
            self._lu = spla.splu(ops.assemble_AAt_blocks(g, S).tocsc())

    def solve(self, b, x0=None):
        g, S = self.g, self.S
        A = lambda v: ops.apply_AAt(g, S, v)
        if self.method == "direct":
            return self._lu.solve(b), 0, 0.0
        if self.method == "cg":
            return cgmod.cg(A, b, self.rtol, self.maxit, x0=x0)
        if self.method == "pcg":
            return cgmod.pcg(A, lambda r: apply_Pinv_fast(g, r), b, self.rtol, self.maxit,
                             x0=x0)
        raise ValueError(self.method)


def cp_step(g: Grid, S: ops.Spatial, st: CPState, V: np.ndarray, m0: np.ndarray,
            proj: Projector, cost: Coupling = LINEAR, u0=None) -> dict:
    """One CP iteration in place; returns per-iteration diagnostics. u0: the
    initial guess of the projection's solve (warm start), else zero."""
    z = st.xi + st.sigma * st.ybar
    b = ops.apply_Cr(g, S, z) - st.sigma * ops.rhs_d(g, m0)
    u, its, relres = proj.solve(b, u0)
    xi_new = ops.apply_CrT(g, S, u)
    y_new = prox_primal(g, st.y - st.tau * xi_new, V, st.tau, cost)
    theta = 1.0 / np.sqrt(1.0 + 2.0 * g.gamma * st.tau)
    ybar = y_new + theta * (y_new - st.y)
    dm = float(np.linalg.norm(y_new[: g.n] - st.y[: g.n]))
    proj_pt = (z - xi_new) / st.sigma
    info = dict(pcg_iters=its, relres=relres, dm=dm, u=u, b=b,
                mass_proj=proj_pt[: g.n].reshape(g.nt, g.M).sum(axis=1))
    st.xi, st.y, st.ybar = xi_new, y_new, ybar
    st.tau, st.sigma, st.theta = theta * st.tau, st.sigma / theta, theta
    st.it += 1
    return info


def cp_solve(g: Grid, V: np.ndarray, m0: np.ndarray, iters: int, method: str = "cg",
             rtol: float = 1e-10, maxit: int = 100000, state: CPState | None = None,
             keep_info: bool = False, cost: Coupling = LINEAR):
    """Run `iters` CP iterations from cp_init (or from `state`). Returns
    (state, list of per-iteration diagnostics)."""
    S = ops.Spatial(g)
    st = state.copy() if state is not None else cp_init(g, m0)
    proj = Projector(g, S, method, rtol, maxit)
    log = []
    for _ in range(iters):
        info = cp_step(g, S, st, V, m0, proj, cost)
        if not keep_info:
            info.pop("u")
            info.pop("b")
        log.append(info)
    return st, log


def cg_tolerance(r_prev: float | None) -> float:
    """Inner tolerance of Section 5 for the next projection from the latest
    CP change r (relative PCG residual): min(1e-4, max(1e-6, 1e-4 r)); with no
    r yet (the first iteration) the loosest value, 1e-4."""
    if r_prev is None:
        return 1e-4
    return min(1e-4, max(1e-6, 1e-4 * r_prev))


def cp_solve_tol(g: Grid, V: np.ndarray, m0: np.ndarray, max_iter: int, cp_tol: float,
                 maxit: int = 100000, state: CPState | None = None,
                 cost: Coupling = LINEAR, warm: bool = False):
    """CP iterations with the stopping and inner-tolerance rules of Section 5:
    iteration l+1 solves its projection by PCG (Algorithms 1+2) to
    cg_tolerance(r_l), r_l = ||m_l - m_{l-1}||_2 of the previous iteration,
    and the loop ends after the first iteration whose r is <= cp_tol (the
    paper takes cp_tol = 1e-4 ||m_0||), or after max_iter iterations. warm:
    each projection's PCG starts from the previous projection's solution (the
    first from zero).
    Returns (state, per-iteration diagnostics with the tolerance used)."""
    S = ops.Spatial(g)
    st = state.copy() if state is not None else cp_init(g, m0)
    log = []
    r_prev = None
    u_prev = None
    for _ in range(max_iter):
        tol = cg_tolerance(r_prev)
        info = cp_step(g, S, st, V, m0, Projector(g, S, "pcg", tol, maxit), cost,
                       u0=u_prev if warm else None)
        u_prev = info["u"]
        info.pop("u")
        info.pop("b")
        info["cg_tol"] = tol
        log.append(info)
        r_prev = info["dm"]
        if r_prev <= cp_tol:
            break
    return st, log
