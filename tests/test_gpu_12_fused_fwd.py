"""The fused preconditioner passes against the separate kernels.

With the mixed precisions, axis 1 of 256 nodes and N_t <= 128, the time GEMM
of the residual and the forward row transforms of Algorithm 2 run as one
kernel (MFG_TUNE fuse_fwd=1, the default); fuse_fwd=0 keeps the separate time
GEMM and row-transform kernels, which the operator parity tests check against
the oracle. The fused kernel scales its operands in the same column groups,
pairs the same rows and runs the same transform arithmetic, so both give the
same bits: checked on P^{-1} r and on whole PCG solves (where the forward pass
also takes the r.r stopping test) for every mixed precision, both boundary
conditions, several N_t (ragged time padding) and operand-scaling group
widths. The same holds for the update inside the forward pass (fuse_upd) and
for the fused inverse pass (fuse_inv: row transforms, inverse time GEMM and
its dot partials).
"""
import numpy as np
import pytest

from _gpu import dev, empty, host, plan_of, say
from paper_2507_01958_amd import workloads as wl

pytestmark = pytest.mark.gpu

PRECISIONS = ["mixed_fp32", "mixed_fp16", "mixed_bf16"]


def _run(monkeypatch, tune, inst, precision, r, b):
    monkeypatch.setenv("MFG_TUNE", tune)
    with plan_of(inst, precision) as P:
        z = empty(r.size)
        from paper_2507_01958_amd import mfg
        mfg.mfg_precond(P, dev(r), z)
        u = empty(r.size)
        st = mfg.mfg_pcg(P, dev(b), u, 1e-9, 60, raise_not_converged=False)
        return host(z), host(u), st


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("bc", ["periodic", "neumann"])
@pytest.mark.parametrize("nx,nt", [(6, 5), (8, 70), (4, 128)])
def test_fused_forward_bitwise(monkeypatch, precision, bc, nx, nt):
    inst = wl.small_instance(71, 2, nx, 256, nt, bc, 0.1)
    n = nt * nx * 256
    rng = np.random.default_rng(72 + nt)
    r = rng.standard_normal(n) * np.exp(rng.uniform(-3, 3, n))
    b = rng.standard_normal(n)
    say(f"fused fwd {precision} {bc} {nx}x256x{nt}")
    z0, u0, s0 = _run(monkeypatch, "fuse_fwd=0", inst, precision, r, b)
    z1, u1, s1 = _run(monkeypatch, "fuse_fwd=1", inst, precision, r, b)
    assert np.array_equal(z0, z1), np.abs(z0 - z1).max()
    assert np.array_equal(u0, u1), np.abs(u0 - u1).max()
    assert s0 == s1


@pytest.mark.parametrize("shape", ["lp_waves=4,lp_cb=1", "lp_waves=8,lp_cb=1",
                                   "lp_waves=8,lp_cb=2"])
def test_fused_forward_scale_groups(monkeypatch, shape):
    # operand scale groups of 64, 128 and 256 columns; the operand magnitudes
    # vary by column so that groups get different scales
    inst = wl.small_instance(73, 2, 4, 256, 37, "neumann", 0.1)
    n = 37 * 4 * 256
    rng = np.random.default_rng(74)
    r = rng.standard_normal(n) * np.exp(rng.uniform(-8, 8, n))
    b = rng.standard_normal(n)
    say(f"fused fwd groups {shape}")
    z0, u0, _ = _run(monkeypatch, shape + ",fuse_fwd=0", inst, "mixed_fp32", r, b)
    z1, u1, _ = _run(monkeypatch, shape + ",fuse_fwd=1", inst, "mixed_fp32", r, b)
    assert np.array_equal(z0, z1), np.abs(z0 - z1).max()
    assert np.array_equal(u0, u1), np.abs(u0 - u1).max()


def _cp(monkeypatch, tune, inst, precision, warm, iters=4):
    from paper_2507_01958_amd import mfg
    monkeypatch.setenv("MFG_TUNE", tune)
    with plan_of(inst, precision) as P:
        mfg.mfg_set_warm_start(P, warm)
        st = mfg.CPState(P)
        mfg.mfg_cp_init(P, st)
        stats = mfg.mfg_cp_solve(P, st, iters, 1e-8, 200)
        return host(st.xi), host(st.y), stats["pcg_iters"]


@pytest.mark.parametrize("precision,warm", [("mixed_fp32", False), ("mixed_fp16", True),
                                            ("mixed_bf16", False)])
def test_fused_update_cp_bitwise(monkeypatch, precision, warm):
    """The conjugate gradient update inside the fused forward pass (fuse_upd=1)
    against its own kernel (fuse_upd=0) over whole CP iterations (standard and
    flexible PCG, cold and warm starts): the same bits, the same PCG counts."""
    inst = wl.small_instance(75, 2, 8, 256, 40, "neumann", 0.05)
    say(f"fused update cp {precision} warm={warm}")
    a = _cp(monkeypatch, "fuse_upd=0", inst, precision, warm)
    b = _cp(monkeypatch, "fuse_upd=1", inst, precision, warm)
    assert list(a[2]) == list(b[2])
    assert np.array_equal(a[0], b[0]), np.abs(a[0] - b[0]).max()
    assert np.array_equal(a[1], b[1]), np.abs(a[1] - b[1]).max()


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("bc", ["periodic", "neumann"])
@pytest.mark.parametrize("nx,nt,waves", [(6, 5, 8), (8, 70, 4), (4, 128, 8)])
def test_fused_inverse_bitwise(monkeypatch, precision, bc, nx, nt, waves):
    """The fused inverse pass (row transforms + inverse time GEMM with the dot
    partials) against the separate kernels with one 16-node tile per wave:
    the same z, the same partials (hence the same PCG iterates)."""
    inst = wl.small_instance(76, 2, nx, 256, nt, bc, 0.1)
    n = nt * nx * 256
    rng = np.random.default_rng(77 + nt)
    r = rng.standard_normal(n) * np.exp(rng.uniform(-3, 3, n))
    b = rng.standard_normal(n)
    say(f"fused inv {precision} {bc} {nx}x256x{nt} waves={waves}")
    shape = f"lp_cb_i=1,lp_waves_i={waves}"
    z0, u0, s0 = _run(monkeypatch, shape + ",fuse_inv=0", inst, precision, r, b)
    z1, u1, s1 = _run(monkeypatch, shape + ",fuse_inv=1", inst, precision, r, b)
    assert np.array_equal(z0, z1), np.abs(z0 - z1).max()
    assert np.array_equal(u0, u1), np.abs(u0 - u1).max()
    assert s0 == s1


@pytest.mark.parametrize("precision,warm", [("mixed_fp32", True), ("mixed_fp16", False)])
def test_fused_passes_cp_bitwise(monkeypatch, precision, warm):
    """Every fused pass on (forward with the update, inverse) against every
    one off, over whole CP iterations."""
    inst = wl.small_instance(78, 2, 8, 256, 40, "periodic", 0.05)
    say(f"fused passes cp {precision} warm={warm}")
    a = _cp(monkeypatch, "fuse_fwd=0,fuse_upd=0,fuse_inv=0", inst, precision, warm)
    b = _cp(monkeypatch, "fuse_fwd=1,fuse_upd=1,fuse_inv=1", inst, precision, warm)
    assert list(a[2]) == list(b[2])
    assert np.array_equal(a[0], b[0]), np.abs(a[0] - b[0]).max()
    assert np.array_equal(a[1], b[1]), np.abs(a[1] - b[1]).max()



@pytest.mark.parametrize("bc_x,bc_y", [("periodic", "neumann"), ("neumann", "periodic")])
@pytest.mark.parametrize("precision", ["mixed_fp32", "mixed_fp16"])
def test_fused_passes_per_axis_boundaries(monkeypatch, bc_x, bc_y, precision):
    """A boundary type per axis (the transform along axis 1 is the one of
    bc_y): every fused pass on against every one off, P^{-1} r and PCG."""
    inst = wl.mixed_instance(81, 8, 256, 21, bc_x, bc_y, 0.05)
    n = 21 * 8 * 256
    rng = np.random.default_rng(82)
    r = rng.standard_normal(n) * np.exp(rng.uniform(-3, 3, n))
    b = rng.standard_normal(n)
    say(f"fused per-axis {precision} {bc_x}/{bc_y}")
    z0, u0, s0 = _run(monkeypatch, "fuse_fwd=0,fuse_upd=0,fuse_inv=0", inst, precision, r, b)
    z1, u1, s1 = _run(monkeypatch, "fuse_fwd=1,fuse_upd=1,fuse_inv=1", inst, precision, r, b)
    assert np.array_equal(z0, z1), np.abs(z0 - z1).max()
    assert np.array_equal(u0, u1), np.abs(u0 - u1).max()
    assert s0 == s1
