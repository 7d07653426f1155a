"""GPU checks of batched solves (mfg_plan_batch / mfg_batch_cp_solve).

A batched run performs, instance by instance, exactly the arithmetic of
mfg_cp_solve on a single plan: the iterates and the PCG iteration counts must
agree BITWISE with separate single-plan runs, whether the steps are replayed
from the recorded HIP graph or launched eagerly, and across several calls
(the graph is recorded once and replayed, with eager work and host
synchronisation between the replays). One instance is also compared with the
oracle (exact projections) as for the single-plan path.
"""
import numpy as np
import pytest

from _gpu import grid_of, host, say
from oracle import cp as ocp
from paper_2507_01958_amd import mfg
from paper_2507_01958_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _instances():
    # uneven sizes, both boundary conditions, several N_t padding classes
    return [wl.small_instance(21, 2, 16, 24, 12, "periodic", 0.05),
            wl.small_instance(22, 2, 32, 18, 20, "neumann", 0.01),
            wl.small_instance(23, 2, 12, 12, 40, "periodic", 0.5),
            wl.small_instance(24, 2, 24, 16, 7, "neumann", 0.1)]


def _problem(inst, precision):
    return mfg.make_problem(inst.d, inst.nx, inst.ny, inst.nt, inst.bc, inst.nu, inst.gamma,
                            l=inst.l, precision=precision, T=inst.T, lo=inst.lo, hi=inst.hi)


def _tensors(inst):
    import torch
    return torch.from_numpy(inst.V).cuda(), torch.from_numpy(inst.m0).cuda()


def _single(inst, precision, chunks, rtol, maxit):
    V, m0 = _tensors(inst)
    P = mfg.mfg_plan(_problem(inst, precision), V, m0)
    st = mfg.CPState(P)
    mfg.mfg_cp_init(P, st)
    its = []
    for k in chunks:
        its += mfg.mfg_cp_solve(P, st, k, rtol, maxit)["pcg_iters"]
    out = (host(st.xi), host(st.y), host(st.ybar), st.sigma, st.tau, its)
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
    out = [(host(s.xi), host(s.y), host(s.ybar), s.sigma, s.tau, [row[i] for row in its])
           for i, s in enumerate(states)]
    B.close()
    return out


@pytest.mark.parametrize("precision", ["mixed_fp32", "mixed_fp16", "fp64"])
@pytest.mark.parametrize("use_graph", [True, False])
def test_batch_bitwise_equals_single(precision, use_graph):
    insts = _instances()
    chunks = [1, 4, 3]  # the graph is recorded in the first call and replayed in later ones
    rtol, maxit = 1e-10, 300
    say(f"batch {precision} graph={use_graph} x{len(insts)}")
    got = _batched(insts, precision, chunks, rtol, maxit, use_graph)
    for inst, b in zip(insts, got):
        ref = _single(inst, precision, chunks, rtol, maxit)
        assert b[5] == ref[5], (inst.name, b[5], ref[5])
        for name, x, y in zip(["xi", "y", "ybar"], b[:3], ref[:3]):
            assert np.array_equal(x, y), (inst.name, name, np.abs(x - y).max())
        assert b[3] == ref[3] and b[4] == ref[4]


def test_batch_matches_oracle():
    insts = _instances()[:2]
    say("batch vs oracle x25")
    got = _batched(insts, "mixed_fp32", [25], 1e-12, 400, True)
    for inst, b in zip(insts, got):
        g = grid_of(inst)
        ref, _ = ocp.cp_solve(g, inst.V, inst.m0, 25, method="direct")
        n = g.n
        for blk in range(1 + g.ncomp):
            r = ref.y[blk * n:(blk + 1) * n]
            err = np.abs(b[1][blk * n:(blk + 1) * n] - r).max() / max(np.abs(r).max(), 1e-300)
            assert err <= 1e-9, (inst.name, blk, err)


def test_batch_rejects_unsupported():
    import torch
    inst = _instances()[0]
    V, m0 = _tensors(inst)
    # above N_t = 128 the batched mixed-precision time GEMM is the streaming one
    long_inst = wl.small_instance(27, 2, 12, 12, 130, "periodic", 0.1)
    Vl, m0l = _tensors(long_inst)
    import os
    old = os.environ.get("MFG_TUNE")
    os.environ["MFG_TUNE"] = "lp_stream=0"
    try:
        with pytest.raises(mfg.MFGError) as e:
            mfg.mfg_plan_batch([_problem(long_inst, "mixed_fp32")], [Vl], [m0l])
        assert e.value.code == 2
    finally:
        if old is None:
            del os.environ["MFG_TUNE"]
        else:
            os.environ["MFG_TUNE"] = old
    with pytest.raises(mfg.MFGError) as e:
        mfg.mfg_plan_batch([_problem(inst, "mixed_fp32"), _problem(inst, "mixed_fp16")],
                           [V, V], [m0, m0])
    assert e.value.code == 1
    torch.cuda.synchronize()


def test_autotune_keeps_results_and_caches(tmp_path, monkeypatch):
    """The tuned launch shapes change only how work is split: the tuned
    preconditioner agrees with the untuned one to rounding (the dot products'
    summation order may change), and the choice is written to MFG_TUNE_CACHE."""
    import torch
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("MFG_TUNE_CACHE", str(cache))
    inst = wl.small_instance(25, 2, 48, 36, 24, "neumann", 0.02)
    say("autotune 48x36x24")
    V, m0 = _tensors(inst)
    r = torch.from_numpy(wl.random_vector(5, inst.n)).cuda()
    for precision in ["fp64", "mixed_fp32"]:
        P0 = mfg.mfg_plan(_problem(inst, precision), V, m0)
        z0 = torch.empty_like(r)
        mfg.mfg_precond(P0, r, z0)
        mfg.mfg_autotune(P0, 2)
        z1 = torch.empty_like(r)
        mfg.mfg_precond(P0, r, z1)
        a, b = host(z0), host(z1)
        # float64: identical per-element arithmetic; float32: the persistent
        # and blocked GEMMs may accumulate in a different order
        tol = 1e-13 if precision == "fp64" else 1e-5
        assert np.abs(a - b).max() <= tol * np.abs(a).max(), precision
        P0.close()
    lines = cache.read_text().split("\n")
    rows = [ln.split() for ln in lines if ln.strip()]
    assert len(rows) == 2 and all(len(x) == 19 for x in rows)
    assert rows[0][:7] == ["2", "48", "36", "24", "1", "0", "1"] and rows[0][7].startswith("gfx")
    assert rows[1][5] == "1"


def test_batch_autotuned_bitwise_equals_single():
    """After mfg_batch_autotune the tuned shapes are cached; single plans made
    afterwards take the same shapes, so batched and single runs still agree
    bitwise."""
    insts = _instances()
    B_args = ([_problem(i, "mixed_fp32") for i in insts],) + tuple(zip(*[_tensors(i) for i in insts]))
    say("batch autotuned x4")
    B = mfg.mfg_plan_batch(*B_args)
    mfg.mfg_batch_autotune(B, 2)
    states = [mfg.CPState(p) for p in B.plans]
    for p, st in zip(B.plans, states):
        mfg.mfg_cp_init(p, st)
    its = mfg.mfg_batch_cp_solve(B, states, 5, 1e-10, 300)
    got = [(host(s.y), [row[i] for row in its]) for i, s in enumerate(states)]
    B.close()
    for inst, (y, it) in zip(insts, got):
        ref = _single(inst, "mixed_fp32", [5], 1e-10, 300)
        assert it == ref[5]
        assert np.array_equal(y, ref[1]), inst.name


def test_batch_with_a_settled_instance():
    """An instance at its fixed point (uniform m0, V = 0) has a zero first
    right-hand side: its PCG ends before any update, u must come back as zero,
    and it must not disturb the other instances of the batch."""
    insts = _instances()[:3]
    flat = wl.small_instance(26, 2, 16, 12, 8, "periodic", 0.1)
    flat.V = np.zeros_like(flat.V)
    flat.m0 = np.ones_like(flat.m0)
    insts.append(flat)
    say("batch with a settled instance")
    # one step: xi' = Cr^T u must be exactly zero for the settled instance
    got = _batched(insts, "mixed_fp32", [1], 1e-10, 300, False)
    assert got[-1][5] == [0]
    assert not np.any(got[-1][0])
    # more steps (graph replays included): still bitwise the single-plan runs
    got = _batched(insts, "mixed_fp32", [1, 3], 1e-10, 300, True)
    for inst, b in zip(insts, got):
        ref = _single(inst, "mixed_fp32", [1, 3], 1e-10, 300)
        assert b[5] == ref[5], (inst.name, b[5], ref[5])
        for x, y in zip(b[:3], ref[:3]):
            assert np.array_equal(x, y), inst.name


def test_fp64_batch_long_horizons():
    """The float64 batched preconditioner takes any N_t (its time GEMM walks the
    k rows in chunks): instances with N_t above 128 and uneven shapes run
    bitwise as single plans, and one matches the oracle's CP with exact
    projections."""
    insts = [wl.small_instance(28, 2, 16, 12, 200, "neumann", 0.05),
             wl.small_instance(29, 2, 12, 18, 130, "periodic", 0.2),
             wl.small_instance(30, 2, 24, 16, 40, "periodic", 0.01)]
    say("fp64 batch long horizons x3")
    got = _batched(insts, "fp64", [2, 3], 1e-12, 400, True)
    for inst, b in zip(insts, got):
        ref = _single(inst, "fp64", [2, 3], 1e-12, 400)
        assert b[5] == ref[5], (inst.name, b[5], ref[5])
        for name, x, y in zip(["xi", "y", "ybar"], b[:3], ref[:3]):
            assert np.array_equal(x, y), (inst.name, name)
    inst, b = insts[1], got[1]
    g = grid_of(inst)
    ref, _ = ocp.cp_solve(g, inst.V, inst.m0, 5, method="direct")
    n = g.n
    for blk in range(1 + g.ncomp):
        r = ref.y[blk * n:(blk + 1) * n]
        err = np.abs(b[1][blk * n:(blk + 1) * n] - r).max() / max(np.abs(r).max(), 1e-300)
        assert err <= 1e-10, (blk, err)


@pytest.mark.parametrize("precision", ["mixed_fp32", "mixed_fp16", "mixed_bf16"])
def test_mixed_batch_long_horizons(precision):
    """Above N_t = 128 the batched low-precision time GEMM streams V through
    LDS as the single-plan one does: batches mixing long and short horizons run
    bitwise as single plans (graph replays included)."""
    insts = [wl.small_instance(31, 2, 16, 12, 200, "neumann", 0.05),
             wl.small_instance(32, 2, 12, 18, 130, "periodic", 0.2),
             wl.small_instance(33, 2, 24, 16, 40, "periodic", 0.01)]
    say(f"{precision} batch long horizons x3")
    got = _batched(insts, precision, [2, 3], 1e-10, 400, True)
    for inst, b in zip(insts, got):
        ref = _single(inst, precision, [2, 3], 1e-10, 400)
        assert b[5] == ref[5], (inst.name, b[5], ref[5])
        for name, x, y in zip(["xi", "y", "ybar"], b[:3], ref[:3]):
            assert np.array_equal(x, y), (inst.name, name)


@pytest.mark.parametrize("precision,use_graph", [("mixed_fp32", True), ("fp64", False)])
def test_batch_tile_queue_bitwise_equals_single(monkeypatch, precision, use_graph):
    """The batched A phase as a persistent grid over a tile queue (MFG_TUNE
    batch_queue=1: resident blocks take instance tiles from a device counter)
    gives the bits of single plans."""
    monkeypatch.setenv("MFG_TUNE", "batch_queue=1")
    insts = _instances()
    chunks = [1, 4, 3]
    rtol, maxit = 1e-10, 300
    say(f"batch tile queue {precision} graph={use_graph} x{len(insts)}")
    got = _batched(insts, precision, chunks, rtol, maxit, use_graph)
    for inst, b in zip(insts, got):
        ref = _single(inst, precision, chunks, rtol, maxit)
        assert b[5] == ref[5], (inst.name, b[5], ref[5])
        for name, x, y in zip(["xi", "y", "ybar"], b[:3], ref[:3]):
            assert np.array_equal(x, y), (inst.name, name, np.abs(x - y).max())
