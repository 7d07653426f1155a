"""Pins of the oracle's Section 5 stopping and inner-tolerance rules.

* The uniform equilibrium (m0 = 1, V = 0) is the known solution: the loop
  stops at the first change below CPtol with m = 1, w = 0 to that scale (the
  iterates approach it geometrically from the initial point).
* The loop stops at the first iteration whose change r is <= CPtol, never
  earlier; every projection meets its own relative tolerance, which lies in
  [1e-6, 1e-4] and is the loosest value on the first iteration.
* Inexact projections stay close to exact ones: after the same number of
  iterations the state agrees with CP using sparse-LU projections to the
  inner tolerances' scale.
"""
import numpy as np

from oracle import cp as ocp
from oracle.grid import Grid
from paper_2507_01958_amd import workloads as wl


def _grid(inst):
    return Grid(d=inst.d, nx=inst.nx, ny=inst.ny, nt=inst.nt, bc=inst.bc, nu=inst.nu, T=inst.T,
                lo=tuple(inst.lo) + (0.0,) * (2 - inst.d), hi=tuple(inst.hi) + (1.0,) * (2 - inst.d),
                l=inst.l, gamma=inst.gamma)


def test_equilibrium_reached_at_the_stopping_scale():
    inst = wl.small_instance(41, 2, 12, 8, 6, "periodic", 0.1)
    g = _grid(inst)
    m0 = np.ones(g.M)
    cp_tol = 1e-4 * np.linalg.norm(m0)
    st, log = ocp.cp_solve_tol(g, np.zeros(g.M), m0, 200, cp_tol)
    dms = [l["dm"] for l in log]
    assert 1 < len(log) < 200
    assert all(d > cp_tol for d in dms[:-1]) and dms[-1] <= cp_tol
    assert np.linalg.norm(st.y[: g.n] - 1.0) <= 10 * cp_tol
    assert np.abs(st.y[g.n:]).max() <= 10 * cp_tol


def test_stopping_rule_and_inner_tolerances():
    inst = wl.small_instance(42, 2, 24, 18, 12, "neumann", 0.05)
    g = _grid(inst)
    cp_tol = 1e-4 * np.linalg.norm(inst.m0)
    st, log = ocp.cp_solve_tol(g, inst.V, inst.m0, 300, cp_tol)
    dms = [l["dm"] for l in log]
    assert 1 < len(log) < 300
    assert all(d > cp_tol for d in dms[:-1]) and dms[-1] <= cp_tol
    tols = [l["cg_tol"] for l in log]
    assert tols[0] == 1e-4
    assert all(1e-6 <= t <= 1e-4 for t in tols)
    assert all(l["relres"] <= l["cg_tol"] for l in log)
    # tightening follows the previous change: smaller change, no looser solve
    for k in range(2, len(log)):
        if dms[k - 1] < dms[k - 2]:
            assert tols[k] <= tols[k - 1]


def test_inexact_projections_track_exact_ones():
    inst = wl.small_instance(43, 2, 12, 12, 8, "periodic", 0.1)
    g = _grid(inst)
    st, log = ocp.cp_solve_tol(g, inst.V, inst.m0, 12, 0.0)
    assert len(log) == 12
    ref, _ = ocp.cp_solve(g, inst.V, inst.m0, 12, method="direct")
    n = g.n
    for blk in range(1 + g.ncomp):
        a, b = st.y[blk * n:(blk + 1) * n], ref.y[blk * n:(blk + 1) * n]
        assert np.abs(a - b).max() <= 1e-3 * np.abs(b).max()


def test_warm_start_keeps_the_iteration_and_saves_pcg_work():
    """Warm-started projections (the previous solution as initial guess) meet
    the same relative tolerances, so the CP iterates stay within the inner
    tolerances' scale of the cold-started ones; they take fewer PCG
    iterations in all."""
    inst = wl.small_instance(44, 2, 16, 12, 10, "neumann", 0.05)
    g = _grid(inst)
    cp_tol = 1e-4 * np.linalg.norm(inst.m0)
    cold, lc = ocp.cp_solve_tol(g, inst.V, inst.m0, 300, cp_tol)
    warm, lw = ocp.cp_solve_tol(g, inst.V, inst.m0, 300, cp_tol, warm=True)
    assert lw[0]["pcg_iters"] == lc[0]["pcg_iters"]        # the first starts from zero
    assert all(l["relres"] <= l["cg_tol"] for l in lw)
    assert sum(l["pcg_iters"] for l in lw) < sum(l["pcg_iters"] for l in lc)
    assert abs(len(lw) - len(lc)) <= 2
    assert np.linalg.norm(warm.y[: g.n] - cold.y[: g.n]) <= 10 * cp_tol
