"""GPU parity for the couplings and the terminal cost of the paper's two
problems (Section 5.1: f = m^2/2 + V; Section 5.2: f = 0 with the terminal cost
g = (m - mbar)/beta, beta = 1e-3, on the Neumann square [-1/2, 1/2]^2), and for
the value function and discrete HJB residual (Section 2, scheme MFG_T^2_h).

* Prox per cell against the oracle: 1e-12 of the cell's input scale (the
  Newton or bracketed-Newton iterates of both sides end within a few ulps of
  the same root).
* CP iterations against the oracle with exact (LU) projections: 1e-10 of each
  block's max norm, or u kappa(A) where larger (the float64 rounding floor of a
  solve with the reduced matrix).
* The Section 5 rules (mfg_cp_solve_tol) on Problem 1 at 16^2 x 128 (the
  smallest shape of Tables 5.1-5.2): the same CP and per-solve PCG counts as
  the oracle.
* Gradients through CP with these costs against the oracle's reverse pass
  (1e-7 normwise, as for the linear coupling).
* Value function: against the oracle's (LU multiplier) on the same state, to
  the same CP bound; HJB residual: against the oracle's formula on the same
  (y, u), 1e-12 of the terms' scale; at converged solutions the residual is at
  rounding level where m > 0 and the flux equals m P_K(-[D_h u]).
"""
import numpy as np
import pytest

from _gpu import dev, empty, fp64_floor, grid_of, host, say
from oracle import adjoint as oadj
from oracle import cp as ocp
from oracle import operators as ops
from oracle import prox as oprox
from oracle import value as oval
from paper_2507_01958_amd import autograd as mad
from paper_2507_01958_amd import mfg
from paper_2507_01958_amd import workloads as wl

pytestmark = pytest.mark.gpu

COUPLING = {0.0: "linear", 0.5: "quadratic"}


def _case(kind, n, nt, nu):
    """(instance, oracle coupling, binding coupling name, beta, mbar or None)."""
    if kind == "problem1":
        return wl.paper_problem1(n, nt, nu), oprox.PROBLEM1, "quadratic", 0.0, None
    if kind == "problem2":
        inst, mbar, beta = wl.paper_problem2(n, nt, nu)
        return inst, oprox.problem2_coupling(mbar, beta), "potential", beta, mbar
    if kind == "cubic_terminal":
        inst = wl.small_instance(907, 2, n, n, nt, "periodic", nu)
        mbar = wl.gaussian_mixture(np.random.default_rng(908), 2, n, n, "periodic", 3)
        cost = oprox.Coupling(c2=0.5, c1=0.0, beta=0.5, mbar_T=mbar)
        return inst, cost, "quadratic", 0.5, mbar
    inst = wl.small_instance(909, 2, n, n, nt, "neumann", nu)
    return inst, oprox.LINEAR, "linear", 0.0, None


def _plan(inst, coupling, beta, mbar, precision="fp64"):
    import torch
    pb = mfg.make_problem(inst.d, inst.nx, inst.ny, inst.nt, inst.bc, inst.nu, inst.gamma,
                          l=inst.l, precision=precision, T=inst.T, lo=inst.lo, hi=inst.hi,
                          coupling=coupling, beta=beta)
    P = mfg.mfg_plan(pb, torch.from_numpy(inst.V).cuda(), torch.from_numpy(inst.m0).cuda())
    if mbar is not None:
        mfg.mfg_set_target(P, dev(mbar))
    return P, pb


def _blocks_err(g, a, ref):
    n = g.n
    return [np.abs(a[b * n:(b + 1) * n] - ref[b * n:(b + 1) * n]).max()
            / max(np.abs(ref[b * n:(b + 1) * n]).max(), 1e-300) for b in range(1 + g.ncomp)]


KINDS = ["problem1", "problem2", "cubic_terminal"]


@pytest.mark.parametrize("kind", KINDS)
def test_prox_with_coupling(kind):
    inst, cost, cname, beta, mbar = _case(kind, 12, 6, 0.1)
    g = grid_of(inst)
    say(f"prox {kind}")
    rng = np.random.default_rng(910)
    v = rng.standard_normal((1 + g.ncomp) * g.n) * 2.0
    P, _ = _plan(inst, cname, beta, mbar)
    for tau in [0.05, 0.7, 3.0]:
        ref = oprox.prox_primal(g, v, inst.V, tau, cost)
        yv = empty(v.size)
        mfg.mfg_prox(P, dev(v), tau, yv)
        got = host(yv)
        c1, Vt = oprox.cell_coefficients(g, inst.V, cost)
        cell = np.abs(v[: g.n]) + tau * np.abs(Vt) + 1.0
        scale = np.tile(cell, 1 + g.ncomp) + np.abs(v)
        err = np.abs(got - ref) / scale
        assert err.max() <= 1e-12, (tau, err.max())
        assert got[: g.n].min() >= 0.0
    P.close()


@pytest.mark.parametrize("kind,n,nt,nu,iters", [("problem1", 16, 16, 0.1, 40),
                                                ("problem2", 12, 16, 0.1, 40),
                                                ("cubic_terminal", 12, 10, 0.05, 40)])
def test_cp_with_coupling(kind, n, nt, nu, iters):
    inst, cost, cname, beta, mbar = _case(kind, n, nt, nu)
    g = grid_of(inst)
    say(f"cp x{iters} {kind} {n}^2x{nt}")
    ref, _ = ocp.cp_solve(g, inst.V, inst.m0, iters, method="direct", cost=cost)
    P, _ = _plan(inst, cname, beta, mbar)
    st = mfg.CPState(P)
    mfg.mfg_cp_init(P, st)
    mfg.mfg_cp_solve(P, st, iters, 1e-13, 500)
    xi, y = host(st.xi), host(st.y)
    P.close()
    errs = _blocks_err(g, y, ref.y) + _blocks_err(g, xi, ref.xi)
    tol = max(1e-10, fp64_floor(g))
    say(f"  max block err {max(errs):.2e} (bound {tol:.2e})")
    assert max(errs) <= tol, errs
    assert y[: g.n].min() >= 0.0


@pytest.mark.parametrize("nu", [1.0, 0.1, 0.01])
def test_problem1_section5_rules_match_oracle(nu):
    inst, cost, cname, beta, mbar = _case("problem1", 16, 128, nu)
    g = grid_of(inst)
    cp_tol = 1e-4 * np.linalg.norm(inst.m0)
    say(f"problem 1 cp_tol nu={nu}")
    ref, log = ocp.cp_solve_tol(g, inst.V, inst.m0, 400, cp_tol, 500, cost=cost)
    P, _ = _plan(inst, cname, beta, mbar)
    st = mfg.CPState(P)
    mfg.mfg_cp_init(P, st)
    out = mfg.mfg_cp_solve_tol(P, st, 400, cp_tol, 500)
    y = host(st.y)
    P.close()
    say(f"  CP iterations gpu {out['n_done']} oracle {len(log)}, avg PCG "
        f"{np.mean(out['pcg_iters']):.2f} / {np.mean([l['pcg_iters'] for l in log]):.2f}")
    assert out["n_done"] == len(log)
    # the uniform m0 is feasible, so the first right-hand side is zero in exact
    # arithmetic: each side solves its own rounding noise there (the GPU's is
    # exactly zero: no iteration); every later solve takes the same count
    assert out["pcg_iters"][0] in (0, log[0]["pcg_iters"])
    assert out["pcg_iters"][1:] == [l["pcg_iters"] for l in log[1:]]
    errs = _blocks_err(g, y, ref.y)
    assert max(errs) <= 1e-9, errs


@pytest.mark.parametrize("kind", ["problem1", "cubic_terminal"])
def test_gradient_with_coupling(kind):
    import torch
    inst, cost, cname, beta, mbar = _case(kind, 8, 6, 0.1)
    if kind == "problem1":
        # a non-uniform m0: from the uniform one the first prox meets wbar = 0
        # exactly, where the prox is not differentiable (the kink of P_K)
        inst.m0 = wl.gaussian_mixture(np.random.default_rng(913), 2, 8, 8, inst.bc, 3)
    g = grid_of(inst)
    mt = wl.gaussian_mixture(np.random.default_rng(911), 2, 8, 8, inst.bc, 3)
    iters = 11
    say(f"gradient {kind}")
    st, _ = ocp.cp_solve(g, inst.V, inst.m0, iters, method="direct", cost=cost)
    _, gy = oadj.terminal_loss_grad(g, st.y, mt)
    gm0_ref, gV_ref, _ = oadj.cp_gradient(g, inst.V, inst.m0, iters, gy, cost=cost)
    pb = mfg.make_problem(inst.d, inst.nx, inst.ny, inst.nt, inst.bc, inst.nu, inst.gamma,
                          T=inst.T, lo=inst.lo, hi=inst.hi, coupling=cname, beta=beta)
    m0 = dev(inst.m0).requires_grad_(True)
    V = dev(inst.V).requires_grad_(True)
    y = mad.cp_solve(pb, m0, V, iters, rtol=1e-12, maxit=500, every=4,
                     mbar=None if mbar is None else dev(mbar))
    loss = 0.5 * ((mad.terminal_m(pb, y) - dev(mt)) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    for got, ref in [(host(m0.grad), gm0_ref), (host(V.grad), gV_ref)]:
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert err <= 1e-7, err


@pytest.mark.parametrize("kind", ["linear", "problem1", "cubic_terminal"])
def test_value_function_and_hjb(kind):
    n, nt = 8, 10
    inst, cost, cname, beta, mbar = _case(kind, n, nt, 0.1)
    g = grid_of(inst)
    S = ops.Spatial(g)
    iters = 400
    say(f"value function + HJB {kind}")
    ref, log = ocp.cp_solve(g, inst.V, inst.m0, iters, method="direct", cost=cost)
    u_ref = oval.value_function(g, S, ref.xi, ref.y, cost)
    P, _ = _plan(inst, cname, beta, mbar)
    st = mfg.CPState(P)
    mfg.mfg_cp_init(P, st)
    mfg.mfg_cp_solve(P, st, iters, 1e-13, 500)
    u = empty((g.nt + 1) * g.M)
    mfg.mfg_value_function(P, st, 1e-13, 500, u)
    R = empty(g.n)
    mfg.mfg_hjb_residual(P, st.y, u, R)
    ug, Rg, yg = host(u).reshape(g.nt + 1, g.M), host(R).reshape(g.nt, g.M), host(st.y)
    # the residual operator on identical inputs
    rng = np.random.default_rng(912)
    ytest = np.abs(rng.standard_normal((1 + g.ncomp) * g.n))
    utest = rng.standard_normal((g.nt + 1) * g.M)
    R2 = empty(g.n)
    mfg.mfg_hjb_residual(P, dev(ytest), dev(utest), R2)
    R2g = host(R2).reshape(g.nt, g.M)
    P.close()
    # value function of the converged state
    tol = max(1e-10, fp64_floor(g))
    assert np.abs(ug - u_ref).max() <= tol * np.abs(u_ref).max()
    # HJB residual operator: same formula, rounding of the terms
    Rref = oval.hjb_residual(g, S, utest.reshape(g.nt + 1, g.M), ytest, inst.V, cost)
    term = (np.abs(utest).max() / g.dt + g.nu * np.abs(utest).max() * 8 / g.dx ** 2
            + np.abs(utest).max() ** 2 / g.dx ** 2 + np.abs(ytest).max() ** 2 + np.abs(inst.V).max())
    assert np.abs(R2g - Rref).max() <= 1e-12 * term
    # the converged GPU solution satisfies the scheme
    m = yg[: g.n].reshape(g.nt, g.M)
    scale = np.abs(ug).max() / g.dt + np.abs(oval.coupling_value(m, inst.V, cost)).max() + 1
    act = m > 0
    assert np.abs(Rg[act]).max() <= 1e-9 * scale
    if (~act).any():
        assert Rg[~act].max() <= 1e-9 * scale
    F = oval.flux_residual(g, S, ug, yg)
    assert np.abs(F).max() <= 1e-9 * (1 + np.abs(yg[g.n:]).max())


def test_set_target_needs_a_terminal_cost():
    inst, cost, cname, beta, mbar = _case("problem1", 8, 4, 0.1)
    P, _ = _plan(inst, cname, 0.0, None)
    with pytest.raises(mfg.MFGError) as e:
        mfg.mfg_set_target(P, dev(inst.m0))
    assert e.value.code == 1
    P.close()


@pytest.mark.parametrize("multi", [False, True])
def test_mass_drift_statistics(multi):
    """The mass drift reported per iteration equals max_t |h^2 sum m^{t+1} -
    h^2 sum m0| computed from the returned state (single-iteration calls), and
    a multi-step call reports the same sequence."""
    inst, cost, cname, beta, mbar = _case("problem2", 12, 8, 0.1)
    g = grid_of(inst)
    say(f"mass drift multi={multi}")
    P, _ = _plan(inst, cname, beta, mbar)
    st = mfg.CPState(P)
    mfg.mfg_cp_init(P, st)
    hd = g.dx * g.dy
    if multi:
        got = mfg.mfg_cp_solve(P, st, 6, 1e-12, 500, mass=True)["mass_drift"]
        P2, _ = _plan(inst, cname, beta, mbar)
        st2 = mfg.CPState(P2)
        mfg.mfg_cp_init(P2, st2)
        ref = [mfg.mfg_cp_solve(P2, st2, 1, 1e-12, 500, mass=True)["mass_drift"][0]
               for _ in range(6)]
        P2.close()
        assert got == ref
    else:
        for _ in range(6):
            d = mfg.mfg_cp_solve(P, st, 1, 1e-12, 500, mass=True)["mass_drift"][0]
            m = host(st.y)[: g.n].reshape(g.nt, g.M)
            expect = hd * np.abs(m.sum(axis=1) - inst.m0.sum()).max()
            assert abs(d - expect) <= 1e-12 * hd * inst.m0.sum()
    P.close()
