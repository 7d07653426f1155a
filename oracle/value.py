"""Value function recovered from the Chambolle-Pock multiplier, and the
residual of the discrete Hamilton-Jacobi-Bellman equation (Section 2, scheme
MFG_T^2_h, and the optimality system of problem VMFG_h).

A solution y = (m, w) of (VMFG_h) (written with the reduced constraint
Cr y = dr of eq. ABC) has a multiplier lambda (one value per cell of the
reduced constraint) with  -Cr^T lambda in the subdifferential of phi at y.
At a fixed point of the CP iteration the dual variable is xi = Cr^T lambda,
so lambda is the least-squares solution of Cr^T lambda = xi, i.e. the solve
A lambda = Cr xi with the matrix of eq. largeA.

Reading that condition cell by cell with u = -lambda gives the first equation
of (MFG_T^2_h) (Hamiltonian |p|^q'/q', eq. power_hamiltonian):
  m-part, m^{k+1} > 0:
    (u^k - u^{k+1})/dt + nu K u^k + |P_K(-[D_h u]^k)|^q' / q' = f(x, m^{k+1})
    for k = 0..N_t-1, with u^{N_t} = g(x, m^{N_t}) (g = 0 without a
    terminal cost: the last constraint row carries no u^{N_t} term, and a
    terminal term G/dt in the objective adds g/dt);
  m^{k+1} = 0: the same expression is <= f(x, 0) (the subdifferential of
    b-hat at (0, 0));
  w-part: w^k = m^{k+1} |P_K(-[D_h u]^k)|^(q'-2) P_K(-[D_h u]^k), the flux of
    the second equation.
In the operators of operators.py, -[D_h u] is B^T u component by component
(B_c^T u along the axis of c: (u_i - u_{i+1})/h for even c, (u_{i-1} - u_i)/h
for odd c, zero across a Neumann boundary).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import operators as ops
from .grid import Grid
from .prox import LINEAR, Coupling, project_cone


def multiplier(g: Grid, S: ops.Spatial, xi: np.ndarray) -> np.ndarray:
    """lambda solving A lambda = Cr xi (sparse LU of eq. largeA; small grids)."""
    A = ops.assemble_AAt_blocks(g, S).tocsc()
    return spla.spsolve(A, ops.apply_Cr(g, S, xi))


def value_function(g: Grid, S: ops.Spatial, xi: np.ndarray, y: np.ndarray,
                   cost: Coupling = LINEAR) -> np.ndarray:
    """u^k, k = 0..N_t, as an (N_t + 1) x M array: u^k = -lambda_k for k < N_t
    and u^{N_t} = g(x, m^{N_t})."""
    lam = multiplier(g, S, xi).reshape(g.nt, g.M)
    u = np.empty((g.nt + 1, g.M))
    u[: g.nt] = -lam
    u[g.nt] = terminal_value(g, y, cost)
    return u


def terminal_value(g: Grid, y: np.ndarray, cost: Coupling = LINEAR) -> np.ndarray:
    """g(x, m^{N_t}) = (m^{N_t} - mbar_T)/beta, or 0 without a terminal cost."""
    if cost.beta <= 0:
        return np.zeros(g.M)
    mT = y[(g.nt - 1) * g.M: g.n]
    return (mT - np.asarray(cost.mbar_T)) / cost.beta


def coupling_value(m: np.ndarray, V: np.ndarray, cost: Coupling = LINEAR) -> np.ndarray:
    """f(x, m) = c2 m^2 + c1 m + V(x)."""
    return cost.c2 * m * m + cost.c1 * m + V


def hjb_residual(g: Grid, S: ops.Spatial, u: np.ndarray, y: np.ndarray, V: np.ndarray,
                 cost: Coupling = LINEAR) -> np.ndarray:
    """R^k = (u^k - u^{k+1})/dt + nu K u^k + |P_K(-[D_h u]^k)|^q'/q' - f(x, m^{k+1})
    for k = 0..N_t-1, as an N_t x M array (zero where m^{k+1} > 0, <= 0 where
    m^{k+1} = 0, at a solution)."""
    m = y[: g.n].reshape(g.nt, g.M)
    R = np.empty((g.nt, g.M))
    qp = cost.qprime
    for k in range(g.nt):
        grad = np.stack([b.T @ u[k] for b in S.B])        # -[D_h u]^k per component
        ham = np.sum(project_cone(grad) ** 2, axis=0) ** (qp / 2.0) / qp
        R[k] = (u[k] - u[k + 1]) / g.dt + g.nu * (S.K @ u[k]) + ham - coupling_value(m[k], V, cost)
    return R


def flux_residual(g: Grid, S: ops.Spatial, u: np.ndarray, y: np.ndarray,
                  cost: Coupling = LINEAR) -> np.ndarray:
    """w^k - m^{k+1} |P_K(-[D_h u]^k)|^(q'-2) P_K(-[D_h u]^k), as a
    (2d) x N_t x M array."""
    nb = 1 + g.ncomp
    Y = y.reshape(nb, g.nt, g.M)
    out = np.empty((g.ncomp, g.nt, g.M))
    qp = cost.qprime
    for k in range(g.nt):
        p = project_cone(np.stack([b.T @ u[k] for b in S.B]))
        norm = np.sqrt(np.sum(p * p, axis=0))
        scale = np.where(norm > 0, norm, 1.0) ** (qp - 2.0) if qp != 2.0 else 1.0
        out[:, k] = Y[1:, k] - Y[0, k][None, :] * scale * p
    return out
