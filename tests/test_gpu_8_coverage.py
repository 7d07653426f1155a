"""GPU parity for configurations the other files do not reach, and the error
statuses of the C ABI.

* Batches with spatial axes of 64, 128, 192 and 256 nodes (the register FFT
  kernels of the batched path and the LDS path at 192) and small N_t: bitwise
  equal to single-plan runs (graph and eager), and within 1e-9 of the oracle.
* A single plan with 192-node axes: preconditioner and PCG against the oracle.
* The 128^2 x 64 torus at the four viscosities 1e-3 .. 1: PCG residuals and two
  CP iterations against the oracle, float64 and the float32 preconditioner.
* The 256^2 x 128 Neumann workload: five CP iterations at PCG rtol 1e-12
  against the oracle's CP (Algorithms 1+2 PCG at rtol 1e-12).
* Long horizons against the oracle's exact (sparse LU) projections.
  Float64 CP parity is 1e-10 of each block's max norm, or u kappa(A) where
  that is larger: a float64 solve with A cannot be more accurate than its
  rounding floor u kappa(A) (kappa from a Gershgorin bound of lambda_max and the
  exact lambda_min), which is 1.4e-9 at 256^2 x 128 and 3.1e-9 at N_t = 4096.
* Failure statuses: MFG_ERR_NOT_CONVERGED with the counts filled,
  MFG_ERR_NONFINITE for a NaN right-hand side and for NaN data, invalid m0,
  and a CP state marked unusable (iter = -1) after a failure inside a
  multi-step call.
"""
import ctypes

import numpy as np
import pytest

from _gpu import dev, empty, fp64_floor, grid_of, host, plan_of, say
from oracle import cp as ocp
from oracle import operators as ops
from oracle import precond as pc
from paper_2507_01958_amd import mfg
from paper_2507_01958_amd import workloads as wl

pytestmark = pytest.mark.gpu

_CACHE = {}


def _problem(inst, precision):
    return mfg.make_problem(inst.d, inst.nx, inst.ny, inst.nt, inst.bc, inst.nu, inst.gamma,
                            l=inst.l, precision=precision, T=inst.T, lo=inst.lo, hi=inst.hi)


def _tensors(inst):
    import torch
    return torch.from_numpy(inst.V).cuda(), torch.from_numpy(inst.m0).cuda()


def _blocks_err(g, a, ref):
    n = g.n
    out = []
    for blk in range(1 + g.ncomp):
        r = ref[blk * n:(blk + 1) * n]
        out.append(np.abs(a[blk * n:(blk + 1) * n] - r).max() / max(np.abs(r).max(), 1e-300))
    return out


# ---------------------------------------------------------------- batches
def _big_axis_instances():
    return [wl.small_instance(801, 2, 64, 128, 12, "periodic", 0.05),
            wl.small_instance(802, 2, 192, 192, 8, "periodic", 0.01),
            wl.small_instance(803, 2, 256, 256, 8, "periodic", 0.2),
            wl.small_instance(804, 2, 128, 64, 16, "neumann", 0.003)]


def _single(inst, precision, chunks, rtol, maxit):
    V, m0 = _tensors(inst)
    P = mfg.mfg_plan(_problem(inst, precision), V, m0)
    st = mfg.CPState(P)
    mfg.mfg_cp_init(P, st)
    its = []
    for k in chunks:
        its += mfg.mfg_cp_solve(P, st, k, rtol, maxit)["pcg_iters"]
    out = (host(st.xi), host(st.y), host(st.ybar), its)
    P.close()
    return out


def _batched(insts, precision, chunks, rtol, maxit, use_graph):
    Vs, m0s = zip(*[_tensors(i) for i in insts])
    B = mfg.mfg_plan_batch([_problem(i, precision) for i in insts], Vs, m0s)
    states = [mfg.CPState(p) for p in B.plans]
    for p, st in zip(B.plans, states):
        mfg.mfg_cp_init(p, st)
    its = []
    for k in chunks:
        its += mfg.mfg_batch_cp_solve(B, states, k, rtol, maxit, use_graph=use_graph)
    out = [(host(s.xi), host(s.y), host(s.ybar), [row[i] for row in its])
           for i, s in enumerate(states)]
    B.close()
    return out


@pytest.mark.parametrize("precision", ["mixed_fp32", "mixed_fp16", "fp64"])
@pytest.mark.parametrize("use_graph", [True, False])
def test_batch_big_axes_bitwise(precision, use_graph):
    insts = _big_axis_instances()
    chunks = [1, 2]
    say(f"batch big axes {precision} graph={use_graph}")
    got = _batched(insts, precision, chunks, 1e-10, 300, use_graph)
    for inst, b in zip(insts, got):
        ref = _single(inst, precision, chunks, 1e-10, 300)
        assert b[3] == ref[3], (inst.name, b[3], ref[3])
        for name, x, y in zip(["xi", "y", "ybar"], b[:3], ref[:3]):
            assert np.array_equal(x, y), (inst.name, name, np.abs(x - y).max())


def test_batch_big_axes_oracle():
    insts = _big_axis_instances()
    say("batch big axes vs oracle x3")
    got = _batched(insts, "mixed_fp32", [3], 1e-12, 400, True)
    for inst, b in zip(insts, got):
        g = grid_of(inst)
        ref, _ = ocp.cp_solve(g, inst.V, inst.m0, 3, method="pcg", rtol=1e-12, maxit=500)
        errs = _blocks_err(g, b[1], ref.y) + _blocks_err(g, b[0], ref.xi)
        floor = fp64_floor(g)
        say(f"  {inst.name}: max block err {max(errs):.2e} (u kappa {floor:.2e})")
        assert max(errs) <= max(1e-9, floor), (inst.name, errs)


# ------------------------------------------------------ single plan, axis 192
@pytest.mark.parametrize("bc", ["periodic", "neumann"])
@pytest.mark.parametrize("precision", ["fp64", "mixed_fp32"])
def test_axis_192_precond_and_pcg(bc, precision):
    inst = wl.small_instance(810, 2, 192, 192, 12, bc, 0.02)
    g = grid_of(inst)
    S = ops.Spatial(g)
    say(f"axis 192 {bc} {precision}")
    r = np.random.default_rng(811).standard_normal(g.n)
    ref = pc.apply_Pinv_fast(g, r)
    with plan_of(inst, precision=precision) as P:
        z = empty(g.n)
        mfg.mfg_precond(P, dev(r), z)
        got = host(z)
        u = empty(g.n)
        its, rel, _ = mfg.mfg_pcg(P, dev(r), u, 1e-10, 200)
        x = host(u)
    if precision == "fp64":
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    else:
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 2e-5
    res = np.linalg.norm(r - ops.apply_AAt(g, S, x))
    floor = np.finfo(float).eps * np.linalg.norm(ops.abs_AAt_bound(g, S, x))
    assert rel <= 2e-10
    assert res <= 2e-10 * np.linalg.norm(r) + 50 * floor


# ------------------------------------------------ 128^2 x 64 torus, nu sweep
NUS = [1e-3, 1e-2, 1e-1, 1.0]


def _c2(nu):
    key = ("c2", nu)
    if key not in _CACHE:
        inst = wl.torus_2d_trig(nu=nu)
        g = grid_of(inst)
        ref, _ = ocp.cp_solve(g, inst.V, inst.m0, 2, method="pcg", rtol=1e-12, maxit=500)
        _CACHE[key] = (inst, g, ref)
    return _CACHE[key]


@pytest.mark.parametrize("precision", ["fp64", "mixed_fp32"])
@pytest.mark.parametrize("nu", NUS)
def test_c2_nu_sweep(nu, precision):
    inst, g, ref = _c2(nu)
    S = ops.Spatial(g)
    say(f"128^2x64 nu={nu} {precision}: pcg + cp x2")
    b = np.random.default_rng(820).standard_normal(g.n)
    rtol_cp, tol = (1e-12, max(1e-10, fp64_floor(g))) if precision == "fp64" else (1e-10, 1e-7)
    with plan_of(inst, precision=precision) as P:
        u = empty(g.n)
        its, rel, _ = mfg.mfg_pcg(P, dev(b), u, 1e-8, 200)
        x = host(u)
        st = mfg.CPState(P)
        mfg.mfg_cp_init(P, st)
        mfg.mfg_cp_solve(P, st, 2, rtol_cp, 500)
        xi, y = host(st.xi), host(st.y)
    res = np.linalg.norm(b - ops.apply_AAt(g, S, x))
    floor = np.finfo(float).eps * np.linalg.norm(ops.abs_AAt_bound(g, S, x))
    assert rel <= 1.01e-8 and res <= 1.01e-8 * np.linalg.norm(b) + 50 * floor
    errs = _blocks_err(g, y, ref.y) + _blocks_err(g, xi, ref.xi)
    say(f"  pcg its {its}, cp max block err {max(errs):.2e}")
    assert max(errs) <= tol, errs


# ----------------------------------------- 256^2 x 128 Neumann, 5 iterations
def _c3_ref():
    if "c3" not in _CACHE:
        inst = wl.neumann_square()
        g = grid_of(inst)
        say("oracle: 5 CP iterations on 256^2x128 (PCG rtol 1e-12)")
        ref, _ = ocp.cp_solve(g, inst.V, inst.m0, 5, method="pcg", rtol=1e-12, maxit=500)
        _CACHE["c3"] = (inst, g, ref)
    return _CACHE["c3"]


def test_c3_five_iterations_fp64():
    inst, g, ref = _c3_ref()
    say("256^2x128 fp64 cp x5 at rtol 1e-12")
    with plan_of(inst) as P:
        mfg.mfg_autotune(P, 1)
        st = mfg.CPState(P)
        mfg.mfg_cp_init(P, st)
        mfg.mfg_cp_solve(P, st, 5, 1e-12, 500)
        xi, y, ybar = host(st.xi), host(st.y), host(st.ybar)
    errs = _blocks_err(g, y, ref.y) + _blocks_err(g, xi, ref.xi) + _blocks_err(g, ybar, ref.ybar)
    floor = fp64_floor(g)
    say(f"  max block err {max(errs):.2e} (u kappa {floor:.2e})")
    assert max(errs) <= max(1e-10, floor), errs


# Errors of each result after 5 CP iterations at the timed PCG tolerance
# (1e-8) against the oracle's iterates (rtol 1e-12), per precision: m, the
# flux blocks w and xi, relative to each block's max norm. The float64 path
# at the same rtol shows the part owed to the tolerance alone (it stops closest
# to 1e-8, in 7 iterations); the mixed modes take 8-20 iterations and end
# further below it. Measured maxima (m, w, xi): fp64 3.7e-9, 6.9e-9, 4.7e-9;
# fp32 2.2e-10, 4.0e-10, 2.4e-10; fp16 2.9e-10, 5.5e-10, 6.1e-10; bf16 2.2e-10,
# 4.8e-11, 2.2e-10. The bounds are these with a margin of about 3.
MIXED_CP_BOUND = {"fp64": 2e-8, "mixed_fp32": 1.2e-9, "mixed_fp16": 2e-9, "mixed_bf16": 7e-10}


@pytest.mark.parametrize("precision", ["fp64", "mixed_fp32", "mixed_fp16", "mixed_bf16"])
def test_c3_per_result_errors(precision):
    inst, g, ref = _c3_ref()
    say(f"256^2x128 {precision} cp x5 at rtol 1e-8: per-result errors")
    with plan_of(inst, precision=precision) as P:
        mfg.mfg_autotune(P, 1)
        st = mfg.CPState(P)
        mfg.mfg_cp_init(P, st)
        mfg.mfg_cp_solve(P, st, 5, 1e-8, 500)
        xi, y = host(st.xi), host(st.y)
    ey = _blocks_err(g, y, ref.y)
    ex = _blocks_err(g, xi, ref.xi)
    say(f"  {precision}: m {ey[0]:.2e} w {max(ey[1:]):.2e} xi_m {ex[0]:.2e} xi_w {max(ex[1:]):.2e}")
    assert max(ey + ex) <= MIXED_CP_BOUND[precision], (ey, ex)


# ---------------------------------------- long horizons against exact solves
LONG_LU = [
    # (d, nx, ny, nt, bc, nu): band-limited A, sparse LU in seconds
    (1, 16, 1, 4096, "neumann", 0.1),
    (1, 32, 1, 300, "periodic", 0.1),
    (1, 8, 1, 2048, "periodic", 0.01),
]


@pytest.mark.parametrize("case", LONG_LU, ids=lambda c: f"d{c[0]}_{c[1]}x{c[2]}x{c[3]}_{c[4]}")
def test_long_cp_against_exact_projections(case):
    d, nx, ny, nt, bc, nu = case
    inst = wl.small_instance(300, d, nx, ny, nt, bc, nu)
    g = grid_of(inst)
    say(f"long cp x3 vs LU {case}")
    ref, _ = ocp.cp_solve(g, inst.V, inst.m0, 3, method="direct")
    with plan_of(inst) as P:
        st = mfg.CPState(P)
        mfg.mfg_cp_init(P, st)
        mfg.mfg_cp_solve(P, st, 3, 1e-14, 800, raise_not_converged=False)
        xi, y = host(st.xi), host(st.y)
    errs = _blocks_err(g, y, ref.y) + _blocks_err(g, xi, ref.xi)
    floor = fp64_floor(g)
    say(f"  max block err {max(errs):.2e} (u kappa {floor:.2e})")
    assert max(errs) <= max(1e-10, floor), errs


# ------------------------------------------------------------ error statuses
def test_status_not_converged_fills_counts():
    inst = wl.small_instance(830, 2, 16, 12, 8, "periodic", 0.1)
    say("status: not converged")
    lib = mfg.load()
    b = dev(wl.random_vector(831, inst.n))
    with plan_of(inst) as P:
        u = empty(inst.n)
        its, rel = ctypes.c_int(-7), ctypes.c_double(-1.0)
        rc = lib.mfg_pcg(P.handle, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                         1e-30, 1, ctypes.byref(its), ctypes.byref(rel))
        assert rc == 3
        assert its.value == 1 and 0.0 < rel.value < 1.0
        assert b"maxit" in lib.mfg_last_error()


def test_status_nonfinite_rhs_and_data():
    import torch
    inst = wl.small_instance(832, 2, 16, 12, 8, "neumann", 0.1)
    say("status: non-finite")
    b = wl.random_vector(833, inst.n)
    b[17] = np.nan
    with plan_of(inst) as P:
        u = empty(inst.n)
        with pytest.raises(mfg.MFGError) as e:
            mfg.mfg_pcg(P, dev(b), u, 1e-8, 50)
        assert e.value.code == 5
        # the plan stays usable after the failure
        its, rel, rc = mfg.mfg_pcg(P, dev(wl.random_vector(834, inst.n)), u, 1e-8, 50)
        assert rc == 0 and rel <= 1.01e-8
    V, m0 = _tensors(inst)
    bad = m0.clone()
    bad[3] = float("nan")
    with pytest.raises(mfg.MFGError) as e:
        mfg.mfg_plan(_problem(inst, "fp64"), V, bad)
    assert e.value.code == 5
    bad = m0.clone()
    bad[3] = -1e-3
    with pytest.raises(mfg.MFGError) as e:
        mfg.mfg_plan(_problem(inst, "fp64"), V, bad)
    assert e.value.code == 1
    badV = V.clone()
    badV[0] = float("inf")
    with pytest.raises(mfg.MFGError) as e:
        mfg.mfg_plan(_problem(inst, "fp64"), badV, m0)
    assert e.value.code == 5
    torch.cuda.synchronize()


def test_state_marked_after_failure_inside_a_call():
    """A NaN in y is met by the second step's right-hand side (the first
    step's prox carries it into z): MFG_ERR_NONFINITE and iter = -1."""
    inst = wl.small_instance(835, 2, 16, 12, 8, "periodic", 0.1)
    say("status: state after a failed multi-step call")
    with plan_of(inst) as P:
        st = mfg.CPState(P)
        mfg.mfg_cp_init(P, st)
        st.y[5] = float("nan")
        with pytest.raises(mfg.MFGError) as e:
            mfg.mfg_cp_solve(P, st, 3, 1e-10, 100)
        assert e.value.code == 5
        assert st.iter == -1
