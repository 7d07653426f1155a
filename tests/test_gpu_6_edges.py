"""GPU parity at the edges of the accepted problems, against the oracle.

* Long horizons, N_t > 128: the time transform leaves the LDS-resident kernels
  for the streaming ones (V through LDS in chunks of 16 or 32 time rows):
  float64 products in FP64, float16 / bfloat16 products (the float32 mode as
  a two-term float16 split) in the MIXED modes. Cases: 200 steps (one full
  and one partial block of 128 output rows, ragged spatial axis 12), the
  N_t = 2048 of the paper's long-horizon runs (Table 5.5), and the largest
  N_t a plan accepts, 4096. Bounds as for the short cases: operator products
  1e-12 of |Op| |x| entrywise, the float64 preconditioner 1e-12 of max |z|,
  the MIXED ones normwise by the arithmetic of each mode (2e-5 with the
  float32 split, 1e-2 float16, 5e-2 bfloat16, as at N_t <= 128), PCG to its
  rtol with the true residual formed by the oracle. CP iterates: both sides
  stop PCG at a 1e-13 relative residual; the bound is 1e-10 of each block's
  max norm, or the float64 rounding floor u kappa(A) of a solve with A where
  that is larger. kappa(A) grows as N_t^2 (lambda_min = lambda_1 / dt^2 stays
  near pi^2 / (4 T^2) while lambda_max ~ 4 / dt^2): u kappa is 3.1e-9 at
  N_t = 4096.
* Zero viscosity with l = 1: the preconditioner of eq. prec is then the
  reduced matrix itself (Section 4.2), so PCG converges in one iteration, to
  the sparse direct solution.
* The smallest horizon a plan accepts, N_t = 2.
"""
import numpy as np
import pytest

from _gpu import dev, empty, fp64_floor, grid_of, host, plan_of, say
from oracle import cp as ocp
from oracle import operators as ops
from oracle import precond as pc
from paper_2507_01958_amd import mfg
from paper_2507_01958_amd import workloads as wl

pytestmark = pytest.mark.gpu

LONG = [
    # (d, nx, ny, nt, bc, nu)
    (1, 32, 1, 300, "periodic", 0.1),
    (2, 16, 12, 200, "neumann", 0.05),
    (2, 16, 16, 2048, "periodic", 0.01),
    (1, 16, 1, 4096, "neumann", 0.1),
]


def _inst(case, seed=0, l=1):
    d, nx, ny, nt, bc, nu = case
    return wl.small_instance(300 + seed, d, nx, ny, nt, bc, nu, l=l)


def _ids(c):
    return f"d{c[0]}_{c[1]}x{c[2]}x{c[3]}_{c[4]}_nu{c[5]}"


@pytest.mark.parametrize("case", LONG, ids=_ids)
def test_long_operators(case):
    inst = _inst(case)
    g = grid_of(inst)
    say(f"long AAt/C/CT {_ids(case)}")
    S = ops.Spatial(g)
    rng = np.random.default_rng(11)
    u = rng.standard_normal(g.n)
    y = rng.standard_normal((1 + g.ncomp) * g.n)
    with plan_of(inst) as P:
        q = empty(g.n)
        mfg.mfg_apply_AAt(P, dev(u), q)
        b = empty(g.n)
        mfg.mfg_apply_C(P, dev(y), b)
        yt = empty((1 + g.ncomp) * g.n)
        mfg.mfg_apply_CT(P, dev(u), yt)
        got_q, got_b, got_y = host(q), host(b), host(yt)
    for got, ref, scale in [
        (got_q, ops.apply_AAt(g, S, u), ops.abs_AAt_bound(g, S, u)),
        (got_b, ops.apply_Cr(g, S, y), ops.abs_Cr_bound(g, S, y)),
        (got_y, ops.apply_CrT(g, S, u), ops.abs_CrT_bound(g, S, u)),
    ]:
        err = np.abs(got - ref)
        assert np.all(err <= 1e-12 * scale + 1e-300), (err / scale).max()


MIXED_TOL = {"mixed_fp32": 2e-5, "mixed_fp16": 1e-2, "mixed_bf16": 5e-2}


@pytest.mark.parametrize("precision", ["fp64", "mixed_fp32", "mixed_fp16", "mixed_bf16"])
@pytest.mark.parametrize("l", [1, 2])
@pytest.mark.parametrize("case", LONG, ids=_ids)
def test_long_precond(case, l, precision):
    inst = _inst(case, l=l)
    g = grid_of(inst, l=l)
    say(f"long precond {precision} l={l} {_ids(case)}")
    r = np.random.default_rng(12).standard_normal(g.n)
    ref = pc.apply_Pinv_fast(g, r)
    with plan_of(inst, precision=precision, l=l) as P:
        z = empty(g.n)
        mfg.mfg_precond(P, dev(r), z)
        got = host(z)
    if precision == "fp64":
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    else:
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        say(f"  normwise error {err:.2e}")
        assert err <= MIXED_TOL[precision], err


@pytest.mark.parametrize("precision", ["mixed_fp32", "mixed_fp16", "mixed_bf16"])
def test_long_lowprec_gemm_against_float64_products(precision, monkeypatch):
    """The streaming low-precision time transform (N_t > 128) against the same
    plan with float64 products there (MFG_TUNE lp_stream=0): the difference is
    the products' rounding only, within each mode's bound."""
    case = (2, 16, 16, 2048, "periodic", 0.01)
    inst = _inst(case)
    g = grid_of(inst)
    say(f"long lp gemm vs f64 products {precision}")
    r = np.random.default_rng(17).standard_normal(g.n)
    out = []
    for lp in ("1", "0"):
        monkeypatch.setenv("MFG_TUNE", f"lp_stream={lp}")
        with plan_of(inst, precision=precision) as P:
            z = empty(g.n)
            mfg.mfg_precond(P, dev(r), z)
            out.append(host(z))
    err = np.linalg.norm(out[0] - out[1]) / np.linalg.norm(out[1])
    say(f"  normwise difference {err:.2e}")
    assert err <= MIXED_TOL[precision], err


@pytest.mark.parametrize("precision", ["fp64", "mixed_fp32", "mixed_fp16"])
@pytest.mark.parametrize("case", LONG, ids=_ids)
def test_long_pcg(case, precision):
    inst = _inst(case)
    g = grid_of(inst)
    say(f"long pcg {precision} {_ids(case)}")
    S = ops.Spatial(g)
    b = np.random.default_rng(13).standard_normal(g.n)
    with plan_of(inst, precision=precision) as P:
        u = empty(g.n)
        its, rel, _ = mfg.mfg_pcg(P, dev(b), u, 1e-10, 300)
        got = host(u)
    assert rel <= 2e-10
    assert its <= (80 if precision == "mixed_fp16" else 40), its
    res = np.linalg.norm(ops.apply_AAt(g, S, got) - b)
    floor = np.finfo(float).eps * np.linalg.norm(ops.abs_AAt_bound(g, S, got))
    assert res <= 2e-10 * np.linalg.norm(b) + 50 * floor, res / np.linalg.norm(b)


def _cp_compare(inst, iters, tol=1e-10):
    g = grid_of(inst)
    tol = max(tol, fp64_floor(g))
    ref, _ = ocp.cp_solve(g, inst.V, inst.m0, iters, method="pcg", rtol=1e-13, maxit=500)
    with plan_of(inst) as P:
        st = mfg.CPState(P)
        mfg.mfg_cp_init(P, st)
        mfg.mfg_cp_solve(P, st, iters, 1e-13, 500)
        xi, y = host(st.xi), host(st.y)
    n = g.n
    for name, a, rb in [("xi", xi, ref.xi), ("y", y, ref.y)]:
        for blk in range(1 + g.ncomp):
            ga, r = a[blk * n:(blk + 1) * n], rb[blk * n:(blk + 1) * n]
            scale = max(np.abs(r).max(), 1e-300)
            assert np.abs(ga - r).max() <= tol * scale, (name, blk, np.abs(ga - r).max() / scale)
    assert y[:n].min() >= 0.0


@pytest.mark.parametrize("case", LONG, ids=_ids)
def test_long_cp(case):
    inst = _inst(case)
    say(f"long cp x3 {_ids(case)}")
    _cp_compare(inst, 3)


@pytest.mark.parametrize("case", [(1, 32, 1, 16, "periodic", 0.0), (2, 24, 18, 7, "neumann", 0.0),
                                  (2, 64, 64, 17, "periodic", 0.0)], ids=_ids)
def test_zero_viscosity_pcg_one_iteration(case):
    import scipy.sparse.linalg as spla
    inst = _inst(case)
    g = grid_of(inst)
    say(f"nu=0 pcg {_ids(case)}")
    b = np.random.default_rng(14).standard_normal(g.n)
    x_ref = spla.spsolve(ops.assemble_AAt_blocks(g).tocsc(), b)
    with plan_of(inst) as P:
        u = empty(g.n)
        its, rel, _ = mfg.mfg_pcg(P, dev(b), u, 1e-8, 50)
        got = host(u)
    assert its == 1
    assert rel <= 1e-8
    assert np.abs(got - x_ref).max() <= 1e-9 * np.abs(x_ref).max()


def test_zero_viscosity_cp():
    inst = _inst((2, 24, 18, 7, "neumann", 0.0))
    say("nu=0 cp x10")
    _cp_compare(inst, 10, 1e-10)


@pytest.mark.parametrize("case", [(1, 16, 1, 2, "neumann", 0.1), (2, 12, 18, 2, "periodic", 0.05)],
                         ids=_ids)
def test_two_time_steps(case):
    inst = _inst(case)
    g = grid_of(inst)
    say(f"nt=2 precond + cp {_ids(case)}")
    r = np.random.default_rng(15).standard_normal(g.n)
    ref = pc.apply_Pinv_fast(g, r)
    with plan_of(inst) as P:
        z = empty(g.n)
        mfg.mfg_precond(P, dev(r), z)
        got = host(z)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    _cp_compare(inst, 5, 1e-10)


@pytest.mark.parametrize("precision", ["fp64", "mixed_fp32"])
def test_long_horizon_autotune_keeps_results(precision, tmp_path, monkeypatch):
    """Autotuning a long-horizon plan (the streaming float64 time kernel, whose
    tuned shape may take two column blocks per wave) changes only how the work
    is split: the tuned preconditioner equals the untuned one to rounding, and
    a CP iteration after tuning still matches the oracle."""
    monkeypatch.setenv("MFG_TUNE_CACHE", str(tmp_path / "tune.txt"))
    case = (2, 16, 16, 2048, "periodic", 0.01)
    inst = _inst(case)
    g = grid_of(inst)
    say(f"long autotune {precision} {_ids(case)}")
    r = np.random.default_rng(16).standard_normal(g.n)
    with plan_of(inst, precision=precision) as P:
        z0 = empty(g.n)
        mfg.mfg_precond(P, dev(r), z0)
        mfg.mfg_autotune(P, 2)
        z1 = empty(g.n)
        mfg.mfg_precond(P, dev(r), z1)
        a, b = host(z0), host(z1)
    assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()
    if precision == "fp64":
        _cp_compare(inst, 2)
