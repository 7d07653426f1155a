"""Reverse-mode derivative of a fixed number of Chambolle-Pock iterations.

The forward map (cp.py, eq. pasosChamPock with the Section 5 schedule) from
(m0, V) to the final primal iterate y_N is differentiated exactly, iteration by
iteration, in reverse. Step l (sigma, tau fixed by the schedule, theta =
(1 + 2 gamma tau)^{-1/2}):

  z = xi + sigma ybar;  b = Cr z - sigma dr(m0);  u = A^{-1} b;  xi' = Cr^T u
  v = y - tau xi';  y' = prox(v; V, tau);  ybar' = y' + theta (y' - y)

Its adjoint, given the adjoints (g_xi', g_y', g_ybar') of the new state:

  g_y'  += (1 + theta) g_ybar';          g_y  = -theta g_ybar'
  g_v    = J_prox(v)^T g_y';             g_V += J_prox,V^T g_y'
  g_y   += g_v;                          g_xi' += -tau g_v
  g_u    = Cr g_xi';   g_b = A^{-1} g_u  (A is symmetric: the same solve)
  g_z    = Cr^T g_b;   g_m0 += -(sigma/dt) g_b[slice 0]   (dr = m0/dt in slice 0)
  g_xi   = g_z;        g_ybar = sigma g_z
and at l = 0, y_0 = ybar_0 = (m0 at every slice, w = 0) adds the m-parts of
g_y_0 + g_ybar_0, summed over slices, to g_m0.

The prox Jacobian follows from the implicit-function theorem on
h'(m) = -a/(2 s^2) + c2 m^2 + (c1 + 1/tau) m + V - mbar/tau = 0 (s = m + tau,
a = |w~|^2, w~ = P_K(wbar); c1, V per cell, the terminal term included on the
last slice), with g = h''(m) = a/s^3 + 2 c2 m + c1 + 1/tau, on the active
branch m > 0:
  dm/dmbar = 1/(tau g),  dm/dV = -1/g,  dm/dwbar_c = chi_c w~_c / (s^2 g),
  w_c = (m/s) w~_c  =>  dw_c = (tau/s^2) w~_c dm + (m/s) chi_c dwbar_c,
with chi_c = 1 when wbar_c lies strictly inside its half-line; every
derivative is zero on the inactive branch (m = 0).
"""
from __future__ import annotations

import numpy as np

from . import operators as ops
from .cp import Projector, cp_init, cp_step
from .grid import Grid
from .prox import LINEAR, Coupling, cell_coefficients, project_cone


def prox_vjp(g: Grid, v: np.ndarray, V: np.ndarray, tau: float, gy: np.ndarray,
             cost: Coupling = LINEAR):
    """J_prox(v)^T gy for a whole primal vector; returns (g_v, g_V (length M)).
    Derived for q' = 2 (the closed-form reduction of the prox)."""
    if cost.qprime != 2.0:
        raise NotImplementedError("the prox derivative is derived for q' = 2")
    from .prox import prox_cells
    nb = 1 + g.ncomp
    c1, Vt = cell_coefficients(g, V, cost)
    vv = v.reshape(nb, -1)
    gyy = gy.reshape(nb, -1)
    m, w = prox_cells(vv[0], vv[1:], Vt, tau, c1=c1, c2=cost.c2)
    wt = project_cone(vv[1:])
    chi = ((wt != 0.0) & (wt == vv[1:])).astype(float)
    a = np.sum(wt * wt, axis=0)
    act = m > 0.0
    s = m + tau
    gpp = a / s ** 3 + 2.0 * cost.c2 * m + c1 + 1.0 / tau
    gm_tot = gyy[0] + np.sum(gyy[1:] * (tau / s ** 2) * wt, axis=0)
    gmb = np.where(act, gm_tot / (tau * gpp), 0.0)
    gVc = np.where(act, -gm_tot / gpp, 0.0)
    gwb = np.where(act[None, :], gm_tot[None, :] * chi * wt / (s ** 2 * gpp)[None, :]
                   + gyy[1:] * (m / s)[None, :] * chi, 0.0)
    gv = np.concatenate([gmb[None], gwb], axis=0).reshape(-1)
    gV = gVc.reshape(g.nt, g.M).sum(axis=0)
    return gv, gV


def forward_record(g: Grid, V, m0, iters, method="direct", rtol=1e-13, maxit=100000,
                   cost: Coupling = LINEAR):
    """Forward CP keeping, per iteration, (sigma, tau, theta, v)."""
    S = ops.Spatial(g)
    st = cp_init(g, m0)
    proj = Projector(g, S, method, rtol, maxit)
    tape = []
    for _ in range(iters):
        sigma, tau, y_old = st.sigma, st.tau, st.y.copy()
        cp_step(g, S, st, V, m0, proj, cost)
        v = y_old - tau * st.xi
        tape.append((sigma, tau, st.theta, v))
    return st, tape, S, proj


def cp_gradient(g: Grid, V, m0, iters, gy_final, method="direct", rtol=1e-13,
                cost: Coupling = LINEAR):
    """Gradient of <gy_final, y_N> with respect to (m0, V)."""
    st, tape, S, proj = forward_record(g, V, m0, iters, method, rtol, cost=cost)
    nb = 1 + g.ncomp
    gxi = np.zeros(nb * g.n)
    gy = np.array(gy_final, dtype=float, copy=True)
    gyb = np.zeros(nb * g.n)
    gm0 = np.zeros(g.M)
    gV = np.zeros(g.M)
    for sigma, tau, theta, v in reversed(tape):
        gy_new = gy + (1.0 + theta) * gyb
        gy_prev = -theta * gyb
        gv, gVl = prox_vjp(g, v, V, tau, gy_new, cost)
        gV += gVl
        gy_prev += gv
        gxi_tot = gxi - tau * gv
        gu = ops.apply_Cr(g, S, gxi_tot)
        gb, _, _ = proj.solve(gu)
        gz = ops.apply_CrT(g, S, gb)
        gm0 += -(sigma / g.dt) * gb[: g.M]
        gxi = gz
        gyb = sigma * gz
        gy = gy_prev
    gm0 += (gy + gyb)[: g.n].reshape(g.nt, g.M).sum(axis=0)
    return gm0, gV, st


def terminal_loss_grad(g: Grid, y: np.ndarray, m_target: np.ndarray):
    """J = 1/2 ||m(., T) - m_target||^2 (plain sum over nodes of the last m
    slice) and dJ/dy."""
    mT = y[(g.nt - 1) * g.M: g.n]
    diff = mT - m_target
    gy = np.zeros_like(y)
    gy[(g.nt - 1) * g.M: g.n] = diff
    return 0.5 * float(diff @ diff), gy
