"""Pins of the value-function recovery and of the Chambolle-Pock solutions
through the discrete HJB equation (Section 2, scheme MFG_T^2_h).

The scheme's first equation is not used by the CP iteration, which only sees
the variational problem (VMFG_h). That a converged CP solution, with the value
function read off its multiplier, satisfies it to rounding is therefore an
independent check of the whole chain: the operators, the prox of each coupling,
the terminal cost and its 1/dt weight, and the iteration's fixed point.

* Uniform equilibrium (closed form): m = 1, w = 0 and u^k = f(1) (N_t - k) dt.
* Converged CP solutions of the linear coupling (Neumann), of Problem 1's
  cubic coupling (periodic) and of a terminal-penalty problem (Neumann): the
  HJB residual is at rounding level where m > 0 and the flux equals
  m P_K(-[D_h u]).
* The residual detects a wrong coupling: evaluated with f = m + V on the cubic
  problem's solution it is of order one.
"""
import numpy as np
import pytest

from oracle import cp
from oracle import operators as ops
from oracle import prox
from oracle import value
from oracle.grid import Grid
from paper_2507_01958_amd import workloads as wl


@pytest.mark.parametrize("cubic", [False, True])
def test_uniform_equilibrium_value_function(cubic):
    g = Grid(d=2, nx=8, ny=4, nt=6, bc="periodic", nu=0.2, T=1.5)
    m0 = np.ones(g.M)
    cost = prox.PROBLEM1 if cubic else prox.LINEAR
    st, _ = cp.cp_solve(g, np.zeros(g.M), m0, 300, method="direct", cost=cost)
    S = ops.Spatial(g)
    u = value.value_function(g, S, st.xi, st.y, cost)
    f1 = 0.5 if cubic else 1.0
    expect = f1 * (g.nt - np.arange(g.nt + 1))[:, None] * g.dt * np.ones((1, g.M))
    assert np.abs(u - expect).max() < 1e-10


def _solve(case):
    if case == "linear_neumann":
        inst = wl.small_instance(3, 2, 8, 6, 10, "neumann", 0.1)
        cost = prox.LINEAR
    elif case == "problem1_periodic":
        inst = wl.paper_problem1(8, 16, 0.1)
        cost = prox.PROBLEM1
    else:
        inst, mbar, _ = wl.paper_problem2(6, 8, 0.5)
        cost = prox.problem2_coupling(mbar, beta=0.5)
    g = Grid(d=2, nx=inst.nx, ny=inst.ny, nt=inst.nt, bc=inst.bc, nu=inst.nu, T=inst.T,
             lo=inst.lo, hi=inst.hi, gamma=inst.gamma)
    st, log = cp.cp_solve(g, inst.V, inst.m0, 400, method="direct", cost=cost)
    return g, inst, cost, st, log


@pytest.mark.parametrize("case", ["linear_neumann", "problem1_periodic", "terminal_neumann"])
def test_cp_solution_satisfies_the_discrete_hjb(case):
    g, inst, cost, st, log = _solve(case)
    assert log[-1]["dm"] < 1e-11
    S = ops.Spatial(g)
    u = value.value_function(g, S, st.xi, st.y, cost)
    R = value.hjb_residual(g, S, u, st.y, inst.V, cost)
    m = st.y[: g.n].reshape(g.nt, g.M)
    scale = np.abs(u).max() / g.dt + np.abs(value.coupling_value(m, inst.V, cost)).max() + 1
    act = m > 0
    assert act.any()
    assert np.abs(R[act]).max() <= 1e-11 * scale
    if (~act).any():
        assert R[~act].max() <= 1e-11 * scale
    F = value.flux_residual(g, S, u, st.y)
    assert np.abs(F).max() <= 1e-11 * (1 + np.abs(st.y[g.n:]).max())
    if cost.beta > 0:
        assert np.allclose(u[-1], (m[-1] - cost.mbar_T) / cost.beta, rtol=0, atol=1e-14)


def test_hjb_residual_detects_a_wrong_coupling():
    g, inst, cost, st, _ = _solve("problem1_periodic")
    S = ops.Spatial(g)
    u = value.value_function(g, S, st.xi, st.y, cost)
    R = value.hjb_residual(g, S, u, st.y, inst.V, prox.LINEAR)
    assert np.abs(R).max() > 0.1
