"""Pins of the oracle's prox and Chambolle-Pock loop.

Prox (Section 3, definition eq. def_prox_operator):
* objective never worse than a bounded quasi-Newton brute-force minimisation
  of the full (m, w) problem (which does not use the derivation);
* wbar = 0 reduces to the scalar quadratic: m = max(0, (mbar - tau V)/(1+tau));
* KKT conditions on the active branch; m >= 0 and w in the cone always.
CP (eq. pasosChamPock, Section 5 schedule):
* uniform equilibrium: periodic torus, m0 = 1 on the unit torus, V = 0 gives
  m = 1, w = 0 (feasible because K 1 = 0, optimal because sum m^2 at fixed mass
  is minimised by the uniform density and b-hat >= 0 vanishes at w = 0);
* the projected point conserves mass dx^d sum_i m_t = dx^d sum_i m0 at every
  time slice up to the solve residual;
* plain CG, preconditioned CG and the direct solve give the same iterates.
"""
import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import cp
from oracle import prox
from oracle.grid import Grid


def _brute(mbar, wbar, V, tau, rng):
    nc = len(wbar)
    best = prox.cell_objective(0.0, np.zeros(nc), mbar, wbar, V, tau)
    sign = np.array([1.0 if c % 2 == 0 else -1.0 for c in range(nc)])

    def obj(x):
        m, w = x[0], x[1:]
        return (w @ w) / (2 * m) + 0.5 * m * m + V * m + ((m - mbar) ** 2 + (w - wbar) @ (w - wbar)) / (2 * tau)

    bounds = [(1e-14, None)] + [((0, None) if s > 0 else (None, 0)) for s in sign]
    for _ in range(4):
        x0 = np.r_[abs(rng.normal()) + 0.1, np.abs(rng.normal(size=nc)) * sign]
        res = minimize(obj, x0, method="L-BFGS-B", bounds=bounds,
                       options=dict(ftol=1e-15, gtol=1e-12, maxiter=5000))
        best = min(best, res.fun)
    return best


@pytest.mark.parametrize("nc", [2, 4])
def test_prox_vs_bruteforce(nc):
    rng = np.random.default_rng(100 + nc)
    for _ in range(60):
        mbar = rng.normal() * 2
        wbar = rng.normal(size=nc) * 2
        V = rng.normal()
        tau = 10 ** rng.uniform(-2, 1)
        m, w = prox.prox_cells(np.array([mbar]), wbar[:, None], np.array([V]), tau)
        ours = prox.cell_objective(m[0], w[:, 0], mbar, wbar, V, tau)
        assert ours <= _brute(mbar, wbar, V, tau, rng) + 1e-10 * (1 + abs(ours))


def test_prox_closed_form_without_flux():
    rng = np.random.default_rng(7)
    mbar = rng.normal(size=500) * 3
    V = rng.normal(size=500)
    for tau in [0.01, 0.7, 5.0]:
        m, w = prox.prox_cells(mbar, np.zeros((4, 500)), V, tau)
        scale = (np.abs(mbar) + tau * np.abs(V)) / (1 + tau)
        err = np.abs(m - np.maximum(0, (mbar - tau * V) / (1 + tau)))
        assert np.all(err <= 4e-16 * scale)
        assert np.all(w == 0)


def test_prox_kkt_and_feasibility():
    rng = np.random.default_rng(9)
    N = 20000
    mbar = rng.normal(size=N) * 2
    wbar = rng.normal(size=(4, N)) * 3
    V = rng.normal(size=N)
    tau = 0.3
    m, w, its = prox.prox_cells(mbar, wbar, V, tau, return_iters=True)
    assert np.all(m >= 0)
    assert np.all(w[0::2] >= 0) and np.all(w[1::2] <= 0)
    assert its.max() <= prox.MAX_NEWTON
    act = m > 0
    # stationarity in m: (mbar - m)/tau = -|w|^2/(2 m^2) + m + V
    a = np.sum(w * w, axis=0)
    res = (mbar - m) / tau - (-a / (2 * np.where(act, m, 1) ** 2) + m + V)
    scale = np.abs(mbar) / tau + np.abs(m) + np.abs(V) + 1
    assert np.abs(res[act] / scale[act]).max() < 1e-12
    # stationarity in w (components inside the cone): (wbar - w)/tau = w/m
    wt = prox.project_cone(wbar)
    inside = (wt != 0) & act[None, :]
    r2 = (wbar - w) / tau - w / np.where(act, m, 1)[None, :]
    assert np.abs(r2[inside]).max() < 1e-10 * (1 + np.abs(wbar).max() / tau)
    # inactive branch criterion
    zero = (2 * tau * tau * V - 2 * tau * mbar - np.sum(wt * wt, axis=0)) >= 0
    assert np.all(m[zero] == 0)


@pytest.mark.parametrize("d", [1, 2])
def test_cp_uniform_equilibrium(d):
    g = Grid(d=d, nx=12, ny=8 if d == 2 else 1, nt=6, bc="periodic", nu=0.1, gamma=5e-4)
    st, log = cp.cp_solve(g, np.zeros(g.M), np.ones(g.M), 400, method="direct")
    assert np.abs(st.y[: g.n] - 1).max() < 1e-10
    assert np.abs(st.y[g.n:]).max() < 1e-10
    assert log[-1]["dm"] < 1e-10


@pytest.mark.parametrize("bc", ["periodic", "neumann"])
def test_cp_projected_mass_and_signs(bc):
    from paper_2507_01958_amd import workloads as wl
    inst = wl.small_instance(21, 2, 8, 6, 5, bc, 0.05)
    g = Grid(d=2, nx=8, ny=6, nt=5, bc=bc, nu=0.05, gamma=inst.gamma)
    st, log = cp.cp_solve(g, inst.V, inst.m0, 30, method="direct")
    mass0 = inst.m0.sum()
    for info in log:
        np.testing.assert_allclose(info["mass_proj"], mass0, rtol=1e-11)
    m = st.y[: g.n]
    w = st.y[g.n:].reshape(4, -1)
    assert np.all(m >= 0) and np.all(w[0::2] >= 0) and np.all(w[1::2] <= 0)


def test_cp_solvers_agree():
    from paper_2507_01958_amd import workloads as wl
    inst = wl.small_instance(31, 1, 16, 1, 8, "periodic", 0.1)
    g = Grid(d=1, nx=16, ny=1, nt=8, bc="periodic", nu=0.1, gamma=inst.gamma)
    ref, _ = cp.cp_solve(g, inst.V, inst.m0, 15, method="direct")
    for method in ["cg", "pcg"]:
        st, _ = cp.cp_solve(g, inst.V, inst.m0, 15, method=method, rtol=1e-14, maxit=5000)
        for a, b in [(st.y, ref.y), (st.xi, ref.xi)]:
            assert np.abs(a - b).max() <= 1e-9 * np.abs(b).max()
