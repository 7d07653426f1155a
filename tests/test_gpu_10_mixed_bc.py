"""GPU parity with a boundary type per axis (d = 2: periodic in one axis,
Neumann in the other; Section 4.3's spatial solver takes a DFT on the periodic
axis and a DCT-II on the Neumann one).

Bounds as for the single-type cases: operator products entrywise within
1e-12 |Op| |x|; P^{-1} normwise within 1e-12 of the oracle's Algorithms 1 + 2
(and the mixed-precision modes within their arithmetic's bound); PCG to the
float64 true residual; 40 CP iterations within 1e-10 of the oracle with exact
projections; batched runs bitwise equal to single-plan runs.
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

CASES = [
    # (nx, ny, nt, bc_x, bc_y, nu): LDS-path axes (ragged), then register-FFT
    # axes of 64, 128 and 256 nodes with a partial last block of lines
    (12, 18, 7, "neumann", "periodic", 0.05),
    (24, 9, 6, "periodic", "neumann", 0.3),
    (64, 36, 5, "periodic", "neumann", 0.02),
    (27, 128, 4, "neumann", "periodic", 0.1),
    (256, 18, 3, "neumann", "periodic", 1e-2),
    (96, 256, 3, "periodic", "neumann", 1.0),
]


def _inst(case, seed=0, l=1):
    nx, ny, nt, bx, by, nu = case
    return wl.mixed_instance(300 + seed, nx, ny, nt, bx, by, nu, l=l)


def _ids(c):
    return f"{c[0]}x{c[1]}x{c[2]}_{c[3][0]}{c[4][0]}_nu{c[5]}"


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_mixed_operators(case):
    inst = _inst(case)
    g = grid_of(inst)
    say(f"mixed AAt/C/CT {_ids(case)}")
    S = ops.Spatial(g)
    rng = np.random.default_rng(1)
    u = rng.standard_normal(g.n)
    y = rng.standard_normal((1 + g.ncomp) * g.n)
    with plan_of(inst) as P:
        q, b, yt = empty(g.n), empty(g.n), empty((1 + g.ncomp) * g.n)
        mfg.mfg_apply_AAt(P, dev(u), q)
        mfg.mfg_apply_C(P, dev(y), b)
        mfg.mfg_apply_CT(P, dev(u), yt)
        got_q, got_b, got_y = host(q), host(b), host(yt)
    for got, ref, scale in [
        (got_q, ops.apply_AAt(g, S, u), ops.abs_AAt_bound(g, S, u)),
        (got_b, ops.apply_Cr(g, S, y), ops.abs_Cr_bound(g, S, y)),
        (got_y, ops.apply_CrT(g, S, u), ops.abs_CrT_bound(g, S, u)),
    ]:
        err = np.abs(got - ref)
        assert np.all(err <= 1e-12 * scale + 1e-300), (err / scale).max()


@pytest.mark.parametrize("l", [1, 2])
@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_mixed_precond(case, l):
    inst = _inst(case, l=l)
    g = grid_of(inst, l=l)
    say(f"mixed precond l={l} {_ids(case)}")
    r = np.random.default_rng(4).standard_normal(g.n)
    ref = pc.apply_Pinv_fast(g, r)
    with plan_of(inst, l=l) as P:
        z = empty(g.n)
        mfg.mfg_precond(P, dev(r), z)
        got = host(z)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("precision,tol", [("mixed_fp32", 2e-5), ("mixed_fp16", 1e-2)])
@pytest.mark.parametrize("case", CASES[2:], ids=_ids)
def test_mixed_precond_low_precision(case, precision, tol):
    inst = _inst(case)
    g = grid_of(inst)
    if precision == "mixed_fp32":
        # float32 spatial solves: each transform leaves an absolute error of
        # order u |r| on every mode, and the modes with the smallest symbol,
        # which dominate P^{-1} r, carry about 1/sqrt(M) of it, so the relative
        # error scales as u sqrt(M) (u = 2^-24)
        tol = max(tol, 8 * 2.0 ** -24 * np.sqrt(g.M))
    say(f"mixed precond {precision} {_ids(case)}")
    r = np.random.default_rng(6).standard_normal(g.n)
    ref = pc.apply_Pinv_fast(g, r)
    with plan_of(inst, precision=precision) as P:
        z = empty(g.n)
        mfg.mfg_precond(P, dev(r), z)
        got = host(z)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= tol


@pytest.mark.parametrize("case", CASES[:4], ids=_ids)
def test_mixed_pcg_true_residual(case):
    import scipy.sparse.linalg as spla
    inst = _inst(case)
    g = grid_of(inst)
    say(f"mixed pcg {_ids(case)}")
    b = np.random.default_rng(5).standard_normal(g.n)
    A = ops.assemble_AAt_blocks(g)
    x_ref = spla.spsolve(A.tocsc(), b)
    with plan_of(inst) as P:
        u = empty(g.n)
        its, rel, _ = mfg.mfg_pcg(P, dev(b), u, 1e-12, 200)
        got = host(u)
    # the true residual has the rounding floor u || |A| |x| || (reached here on
    # the finer axes with N_t = 4, where kappa(A) is large), the solution the
    # floor u kappa(A)
    nb = np.linalg.norm(b)
    floor = np.finfo(float).eps * np.linalg.norm(abs(A) @ np.abs(got))
    assert its <= 40
    assert rel * nb <= 2e-12 * nb + 50 * floor, (rel, floor / nb)
    assert np.linalg.norm(A @ got - b) <= 2e-12 * nb + 50 * floor
    tol = max(1e-9, fp64_floor(g))
    assert np.abs(got - x_ref).max() <= tol * np.abs(x_ref).max()


@pytest.mark.parametrize("case", CASES[:2], ids=_ids)
def test_mixed_cp(case):
    inst = _inst(case)
    g = grid_of(inst)
    say(f"mixed cp x40 {_ids(case)}")
    ref, _ = ocp.cp_solve(g, inst.V, inst.m0, 40, method="direct")
    with plan_of(inst) as P:
        st = mfg.CPState(P)
        mfg.mfg_cp_init(P, st)
        mfg.mfg_cp_solve(P, st, 40, 1e-12, 500)
        n = g.n
        for name, a, b in [("xi", host(st.xi), ref.xi), ("y", host(st.y), ref.y)]:
            for blk in range(1 + g.ncomp):
                rb = b[blk * n:(blk + 1) * n]
                err = np.abs(a[blk * n:(blk + 1) * n] - rb).max() / max(np.abs(rb).max(), 1e-300)
                assert err <= 1e-10, (name, blk, err)


def test_mixed_batch_bitwise_equals_single():
    import torch
    insts = [_inst(CASES[0]), _inst(CASES[1], seed=1),
             wl.small_instance(31, 2, 16, 12, 7, "periodic", 0.05)]
    say("mixed batch x3")

    def problem(inst):
        return mfg.make_problem(2, inst.nx, inst.ny, inst.nt, inst.bc, inst.nu, inst.gamma,
                                l=inst.l, precision="mixed_fp32", T=inst.T, lo=inst.lo,
                                hi=inst.hi)

    Vs = [torch.from_numpy(i.V).cuda() for i in insts]
    m0s = [torch.from_numpy(i.m0).cuda() for i in insts]
    B = mfg.mfg_plan_batch([problem(i) for i in insts], Vs, m0s)
    states = [mfg.CPState(p) for p in B.plans]
    for p, st in zip(B.plans, states):
        mfg.mfg_cp_init(p, st)
    its = mfg.mfg_batch_cp_solve(B, states, 5, 1e-10, 300)
    got = [(host(s.y), [row[i] for row in its]) for i, s in enumerate(states)]
    B.close()
    for inst, V, m0, (y, it) in zip(insts, Vs, m0s, got):
        P = mfg.mfg_plan(problem(inst), V, m0)
        st = mfg.CPState(P)
        mfg.mfg_cp_init(P, st)
        ref_its = mfg.mfg_cp_solve(P, st, 5, 1e-10, 300)["pcg_iters"]
        assert it == ref_its
        assert np.array_equal(y, host(st.y)), inst.name
        P.close()


def test_per_axis_bc_rejected_in_one_dimension():
    import torch
    pb = mfg.make_problem(1, 16, 1, 4, ("periodic", "neumann"), 0.1, 5e-4)
    V = torch.zeros(16, dtype=torch.float64, device="cuda")
    with pytest.raises(mfg.MFGError) as e:
        mfg.mfg_plan(pb, V, V + 1.0)
    assert e.value.code == 1
