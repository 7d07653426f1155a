"""GPU parity at the full workload sizes, element by element against the oracle.

The oracle's slice-wise operators, Algorithm 1+2 preconditioner and vectorised
prox handle the full grids in seconds, so every output is compared, not a
sample:

* 256^2 x 128 Neumann (nu = 1e-2), the timed workload, with the launch shapes
  the timed run uses (mfg_autotune, effort 1);
* 128^2 x 64 periodic (nu = 1e-2) and 256^2 x 100 periodic (nu = 5e-2), the
  other two full-size single-problem workloads, with the default shapes.

Tolerances are those of the small-grid tests (derived there): operators
1e-12 of |Op||x| entrywise, prox 1e-12 of its input scale per cell, float64
preconditioner 1e-12 of max|P^{-1} r|, mixed preconditioners normwise by the
arithmetic of each mode. PCG solves are checked through the residual the
oracle's operator computes for the GPU's solution, and two CP iterations
against the oracle's CP with its own PCG.
"""
import numpy as np
import pytest

from _gpu import dev, empty, grid_of, host, plan_of, say
from oracle import cp as ocp
from oracle import operators as ops
from oracle import precond as pc
from oracle import prox as oprox
from paper_2507_01958_amd import mfg
from paper_2507_01958_amd import workloads as wl

pytestmark = pytest.mark.gpu

MIXED_TOL = {"mixed_fp32": 2e-5, "mixed_fp16": 1e-2, "mixed_bf16": 5e-2}
PRECISIONS = ["fp64"] + list(MIXED_TOL)

_INST = {}


def _workload(name):
    if name not in _INST:
        if name == "neumann256x256x128":
            _INST[name] = wl.neumann_square()
        elif name == "periodic128x128x64":
            _INST[name] = wl.torus_2d_trig()
        else:
            _INST[name] = wl.gradient_instance()[0]
    return _INST[name]


WORKLOADS = ["neumann256x256x128", "periodic128x128x64", "periodic256x256x100"]


def _plan(name, precision="fp64"):
    inst = _workload(name)
    P = plan_of(inst, precision=precision)
    if name == "neumann256x256x128":
        mfg.mfg_autotune(P, 1)  # the timed run's launch shapes
    return P


@pytest.mark.parametrize("name", WORKLOADS)
def test_full_operators(name):
    inst = _workload(name)
    g = grid_of(inst)
    say(f"full operators {name}")
    S = ops.Spatial(g)
    rng = np.random.default_rng(11)
    u = rng.standard_normal(g.n)
    y = rng.standard_normal((1 + g.ncomp) * g.n)
    with _plan(name) as P:
        q, b, yt = empty(g.n), empty(g.n), empty((1 + g.ncomp) * g.n)
        mfg.mfg_apply_AAt(P, dev(u), q)
        mfg.mfg_apply_C(P, dev(y), b)
        mfg.mfg_apply_CT(P, dev(u), yt)
        got = [host(q), host(b), host(yt)]
    refs = [(ops.apply_AAt(g, S, u), ops.abs_AAt_bound(g, S, u)),
            (ops.apply_Cr(g, S, y), ops.abs_Cr_bound(g, S, y)),
            (ops.apply_CrT(g, S, u), ops.abs_CrT_bound(g, S, u))]
    for what, x, (ref, scale) in zip(["AAt", "Cr", "CrT"], got, refs):
        err = np.abs(x - ref)
        assert np.all(err <= 1e-12 * scale + 1e-300), (what, (err / scale).max())


@pytest.mark.parametrize("name", WORKLOADS)
def test_full_prox(name):
    inst = _workload(name)
    g = grid_of(inst)
    say(f"full prox {name}")
    v = np.random.default_rng(12).standard_normal((1 + g.ncomp) * g.n) * 2.0
    tau = 0.3
    ref = oprox.prox_primal(g, v, inst.V, tau)
    with _plan(name) as P:
        yv = empty(v.size)
        mfg.mfg_prox(P, dev(v), tau, yv)
        got = host(yv)
    Vt = np.tile(inst.V, g.nt)
    scale = np.tile(np.abs(v[: g.n]) + tau * np.abs(Vt) + 1.0, 1 + g.ncomp) + np.abs(v)
    assert np.all(np.abs(got - ref) <= 1e-12 * scale)
    assert np.all(got[: g.n] >= 0)


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("name", WORKLOADS)
def test_full_precond(name, precision):
    inst = _workload(name)
    g = grid_of(inst)
    say(f"full precond {name} {precision}")
    r = np.random.default_rng(13).standard_normal(g.n)
    ref = pc.apply_Pinv_fast(g, r)
    with _plan(name, precision) as P:
        z = empty(g.n)
        mfg.mfg_precond(P, dev(r), z)
        got = host(z)
    if precision == "fp64":
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    else:
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert err <= MIXED_TOL[precision], err


def _first_cp_rhs(inst, g, S):
    """Right-hand side of the first projection from the initial point:
    Cr ybar0 - dr with ybar0 = (m0 at every slice, w = 0), xi0 = 0, sigma0 = 1."""
    st = ocp.cp_init(g, inst.m0)
    return ops.apply_Cr(g, S, st.xi + st.ybar) - ops.rhs_d(g, inst.m0)


@pytest.mark.parametrize("precision", PRECISIONS)
def test_full_pcg_residual(precision):
    """PCG to rtol 1e-8 (the timed setting) on the timed workload: the
    residual of the GPU's solution, computed by the oracle's operator, is
    within the tolerance (plus the float64 rounding floor of the check)."""
    name = "neumann256x256x128"
    inst = _workload(name)
    g = grid_of(inst)
    S = ops.Spatial(g)
    say(f"full pcg {precision}")
    rhs = [_first_cp_rhs(inst, g, S), np.random.default_rng(14).standard_normal(g.n)]
    with _plan(name, precision) as P:
        for b in rhs:
            u = empty(g.n)
            its, rel, _ = mfg.mfg_pcg(P, dev(b), u, 1e-8, 200)
            x = host(u)
            res = np.linalg.norm(b - ops.apply_AAt(g, S, x))
            floor = np.finfo(float).eps * np.linalg.norm(ops.abs_AAt_bound(g, S, x))
            assert res <= 1.01e-8 * np.linalg.norm(b) + 50 * floor, (its, res / np.linalg.norm(b))
            assert rel <= 1.01e-8
            assert its <= (40 if precision == "mixed_bf16" else 15), its


@pytest.mark.parametrize("precision,rtol,tol", [("fp64", 1e-12, 1e-9), ("mixed_fp32", 1e-10, 1e-7)])
def test_full_cp_two_iterations(precision, rtol, tol):
    """Two CP iterations on the timed workload against the oracle's CP with
    its own PCG (Algorithms 1+2, rtol 1e-12): both projections are inexact,
    so the iterates agree to the solve tolerance amplified by the operator."""
    name = "neumann256x256x128"
    inst = _workload(name)
    g = grid_of(inst)
    say(f"full cp x2 {precision}")
    if "cp2" not in _INST:
        _INST["cp2"] = ocp.cp_solve(g, inst.V, inst.m0, 2, method="pcg", rtol=1e-12)[0]
    ref = _INST["cp2"]
    with _plan(name, precision) as P:
        st = mfg.CPState(P)
        mfg.mfg_cp_init(P, st)
        mfg.mfg_cp_solve(P, st, 2, rtol, 500)
        got = {"xi": host(st.xi), "y": host(st.y), "ybar": host(st.ybar)}
        assert abs(st.tau - ref.tau) <= 1e-15 * ref.tau
        assert abs(st.sigma - ref.sigma) <= 1e-15 * ref.sigma
    n = g.n
    for key, r in [("xi", ref.xi), ("y", ref.y), ("ybar", ref.ybar)]:
        for blk in range(1 + g.ncomp):
            a, c = got[key][blk * n:(blk + 1) * n], r[blk * n:(blk + 1) * n]
            err = np.abs(a - c).max() / max(np.abs(c).max(), 1e-300)
            assert err <= tol, (key, blk, err)
    assert got["y"][:n].min() >= 0.0
