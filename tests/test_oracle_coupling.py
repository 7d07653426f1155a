"""Pins of the oracle's general coupling and terminal cost (Section 2.1 costs,
the two problems of Section 5).

* The prox with a cubic F (f = c2 m^2 + c1 m + V, c2 > 0) is never worse than
  a bounded quasi-Newton minimisation of the full (m, w) problem, which does
  not use the derivation; with wbar = 0 it is the non-negative root of the
  quadratic stationarity condition, taken from numpy's polynomial root finder;
  its KKT residuals vanish.
* The terminal cost g = (m - mbar_T)/beta changes only the last time slice,
  by 1/(beta dt) in the linear coefficient and -mbar_T/(beta dt) in V.
* Uniform equilibria: f = m^2/2 with V = 0, and a terminal target equal to
  the uniform m0, keep m = 1, w = 0 (Jensen: the uniform density minimises
  sum F(m) at fixed mass; G is minimal at m = mbar_T).
"""
import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import cp
from oracle import prox
from oracle.grid import Grid


def _brute(mbar, wbar, V, tau, c1, c2, rng):
    nc = len(wbar)
    best = prox.cell_objective(0.0, np.zeros(nc), mbar, wbar, V, tau, c1, c2)
    sign = np.array([1.0 if c % 2 == 0 else -1.0 for c in range(nc)])

    def obj(x):
        m, w = x[0], x[1:]
        F = c2 * m ** 3 / 3 + 0.5 * c1 * m * m + V * m
        return (w @ w) / (2 * m) + F + ((m - mbar) ** 2 + (w - wbar) @ (w - wbar)) / (2 * tau)

    bounds = [(1e-14, None)] + [((0, None) if s > 0 else (None, 0)) for s in sign]
    for _ in range(4):
        x0 = np.r_[abs(rng.normal()) + 0.1, np.abs(rng.normal(size=nc)) * sign]
        res = minimize(obj, x0, method="L-BFGS-B", bounds=bounds,
                       options=dict(ftol=1e-15, gtol=1e-12, maxiter=5000))
        best = min(best, res.fun)
    return best


@pytest.mark.parametrize("nc", [2, 4])
def test_cubic_prox_vs_bruteforce(nc):
    rng = np.random.default_rng(300 + nc)
    for _ in range(60):
        mbar = rng.normal() * 2
        wbar = rng.normal(size=nc) * 2
        V = rng.normal()
        tau = 10 ** rng.uniform(-2, 1)
        c2 = 10 ** rng.uniform(-1, 1)
        c1 = rng.choice([0.0, 1.0, 10 ** rng.uniform(-1, 3)])
        m, w = prox.prox_cells(np.array([mbar]), wbar[:, None], np.array([V]), tau,
                               c1=c1, c2=c2)
        ours = prox.cell_objective(m[0], w[:, 0], mbar, wbar, V, tau, c1, c2)
        assert ours <= _brute(mbar, wbar, V, tau, c1, c2, rng) + 1e-10 * (1 + abs(ours))


def test_cubic_prox_without_flux_is_the_quadratic_root():
    rng = np.random.default_rng(17)
    for _ in range(300):
        mbar, V = rng.normal() * 3, rng.normal()
        tau = 10 ** rng.uniform(-2, 1)
        c2, c1 = 10 ** rng.uniform(-2, 1), rng.choice([0.0, 1.0, 37.0])
        m, w = prox.prox_cells(np.array([mbar]), np.zeros((4, 1)), np.array([V]), tau,
                               c1=c1, c2=c2)
        roots = np.roots([c2, c1 + 1.0 / tau, V - mbar / tau])
        pos = [r.real for r in roots if abs(r.imag) < 1e-12 and r.real > 0]
        expect = max(pos) if pos else 0.0
        assert abs(m[0] - expect) <= 1e-12 * (1 + abs(expect))
        assert np.all(w == 0)


def test_cubic_prox_kkt():
    rng = np.random.default_rng(19)
    N = 20000
    mbar = rng.normal(size=N) * 2
    wbar = rng.normal(size=(4, N)) * 3
    V = rng.normal(size=N)
    c1 = np.where(rng.uniform(size=N) < 0.5, 0.0, 50.0)
    tau, c2 = 0.3, 0.5
    m, w, its = prox.prox_cells(mbar, wbar, V, tau, return_iters=True, c1=c1, c2=c2)
    assert np.all(m >= 0)
    assert np.all(w[0::2] >= 0) and np.all(w[1::2] <= 0)
    assert its.max() <= prox.MAX_SAFE_NEWTON
    act = m > 0
    a = np.sum(w * w, axis=0)
    mm = np.where(act, m, 1)
    # stationarity in m: (mbar - m)/tau = -|w|^2/(2 m^2) + c2 m^2 + c1 m + V
    res = (mbar - m) / tau - (-a / (2 * mm ** 2) + c2 * m * m + c1 * m + V)
    scale = np.abs(mbar) / tau + c2 * m * m + c1 * m + np.abs(V) + 1
    assert np.abs(res[act] / scale[act]).max() < 1e-12
    wt = prox.project_cone(wbar)
    inside = (wt != 0) & act[None, :]
    r2 = (wbar - w) / tau - w / mm[None, :]
    assert np.abs(r2[inside]).max() < 1e-10 * (1 + np.abs(wbar).max() / tau)
    zero = (2 * tau * tau * V - 2 * tau * mbar - np.sum(wt * wt, axis=0)) >= 0
    assert np.all(m[zero] == 0) and np.all(m[~zero] > 0)


def test_default_coupling_is_unchanged():
    """c2 = 0, c1 = 1 keeps the linear coupling's monotone Newton bit for bit."""
    rng = np.random.default_rng(23)
    mbar = rng.normal(size=4000)
    wbar = rng.normal(size=(4, 4000))
    V = rng.normal(size=4000)
    a = prox.prox_cells(mbar, wbar, V, 0.7)
    b = prox.prox_cells(mbar, wbar, V, 0.7, c1=np.ones(4000), c2=0.0)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_terminal_cost_changes_only_the_last_slice():
    g = Grid(d=2, nx=4, ny=6, nt=5, bc="neumann", nu=0.1, T=2.0)
    rng = np.random.default_rng(3)
    V = rng.normal(size=g.M)
    mbar_T = rng.uniform(size=g.M)
    cost = prox.Coupling(c2=0.5, c1=0.25, beta=0.01, mbar_T=mbar_T)
    c1, Vt = prox.cell_coefficients(g, V, cost)
    c1 = c1.reshape(g.nt, g.M)
    Vt = Vt.reshape(g.nt, g.M)
    w = 1.0 / (0.01 * (2.0 / 5))
    assert np.all(c1[:-1] == 0.25) and np.allclose(c1[-1], 0.25 + w, rtol=1e-15)
    assert np.all(Vt[:-1] == V[None, :])
    assert np.allclose(Vt[-1], V - w * mbar_T, rtol=1e-14, atol=1e-12)
    c1n, Vn = prox.cell_coefficients(g, V, prox.LINEAR)
    assert np.all(c1n == 1.0) and np.array_equal(Vn, np.tile(V, g.nt))


@pytest.mark.parametrize("terminal", [False, True])
def test_uniform_equilibrium_with_cubic_coupling(terminal):
    g = Grid(d=2, nx=8, ny=6, nt=5, bc="periodic", nu=0.1, gamma=5e-4)
    m0 = np.ones(g.M)
    cost = prox.Coupling(c2=0.5, c1=0.0, beta=1.0 if terminal else 0.0,
                         mbar_T=m0 if terminal else None)
    st, log = cp.cp_solve(g, np.zeros(g.M), m0, 300, method="direct", cost=cost)
    assert np.abs(st.y[: g.n] - 1).max() < 1e-10
    assert np.abs(st.y[g.n:]).max() < 1e-10
