"""Pins of the oracle's reverse pass through the Chambolle-Pock iterations.

* prox_vjp equals the transpose of a central finite-difference Jacobian of the
  per-cell prox (both branches);
* the gradient of J = 1/2 ||m(., T) - m_target||^2 with respect to m0 and V
  equals central finite differences of the oracle's own forward map with exact
  (LU) projections, on random directions.
"""
import numpy as np
import pytest

from oracle import adjoint as adj
from oracle import cp as ocp
from oracle import prox
from oracle.grid import Grid
from paper_2507_01958_amd import workloads as wl


def test_prox_vjp_matches_fd_jacobian():
    g = Grid(d=2, nx=4, ny=4, nt=2, bc="periodic", nu=0.1)
    rng = np.random.default_rng(0)
    v = rng.standard_normal(5 * g.n) * 1.5
    V = rng.standard_normal(g.M) * 0.5
    tau = 0.4
    gy = rng.standard_normal(5 * g.n)
    gv, gV = adj.prox_vjp(g, v, V, tau, gy)
    h = 1e-7
    # directional check on several random directions
    for _ in range(5):
        e = rng.standard_normal(v.size)
        fd = (prox.prox_primal(g, v + h * e, V, tau) - prox.prox_primal(g, v - h * e, V, tau)) / (2 * h)
        assert abs(fd @ gy - gv @ e) <= 1e-6 * (abs(gv @ e) + 1e-3)
        eV = rng.standard_normal(g.M)
        fdV = (prox.prox_primal(g, v, V + h * eV, tau) - prox.prox_primal(g, v, V - h * eV, tau)) / (2 * h)
        assert abs(fdV @ gy - gV @ eV) <= 1e-6 * (abs(gV @ eV) + 1e-3)


@pytest.mark.parametrize("case", [(2, "periodic"), (2, "neumann"), (1, "periodic")])
def test_gradient_matches_finite_differences(case):
    d, bc = case
    inst = wl.small_instance(3, d, 8, 6 if d == 2 else 1, 5, bc, 0.1)
    g = Grid(d=d, nx=inst.nx, ny=inst.ny, nt=inst.nt, bc=bc, nu=inst.nu, gamma=inst.gamma)
    mt = wl.gaussian_mixture(np.random.default_rng(9), d, inst.nx, inst.ny, bc, 3)
    iters = 12
    st, _ = ocp.cp_solve(g, inst.V, inst.m0, iters, method="direct")
    _, gy = adj.terminal_loss_grad(g, st.y, mt)
    gm0, gV, _ = adj.cp_gradient(g, inst.V, inst.m0, iters, gy)
    rng = np.random.default_rng(1)
    h = 1e-6
    for which, grad in [("m0", gm0), ("V", gV)]:
        e = rng.standard_normal(g.M)

        def J(x):
            m0 = inst.m0 + (x * e if which == "m0" else 0.0)
            V = inst.V + (x * e if which == "V" else 0.0)
            s, _ = ocp.cp_solve(g, V, m0, iters, method="direct")
            return adj.terminal_loss_grad(g, s.y, mt)[0]

        fd = (J(h) - J(-h)) / (2 * h)
        an = grad @ e
        assert abs(fd - an) <= 1e-5 * abs(an) + 1e-9, (fd, an)
