"""Pins of the oracle's preconditioner (Section 4).

* V is orthonormal and symmetric and V D_tt V^T = diag(lambda_k) (eq. eigs).
* The DST-I transform equals SciPy's orthonormal DST type I (library routine).
* eq. prec (A with the first block changed) equals the Kronecker form.
* Algorithms 1+2 reproduce a sparse direct solve with the assembled P.
* Lemma 1: P^{-1} A has the eigenvalue 1 with multiplicity >= (N_t - 1) M;
  with l = 1 the spectrum lies in [1, inf), with l = 2 in (0, 1].
* nu = 0 and l = 1 make P equal A (Section 4.2), so PCG stops after 1 step.
"""
import numpy as np
import pytest
import scipy.fft as sfft

from oracle import cg as cgmod
from oracle import operators as ops
from oracle import precond as pc
from oracle.grid import Grid


@pytest.mark.parametrize("l", [1, 2])
@pytest.mark.parametrize("nt", [2, 5, 16, 33])
def test_time_transform_diagonalises_Dtt(l, nt):
    V = pc.time_transform(nt, l)
    np.testing.assert_allclose(V @ V.T, np.eye(nt), atol=1e-13)
    np.testing.assert_allclose(V, V.T, rtol=0, atol=1e-14)
    D = pc.Dtt(nt, l)
    np.testing.assert_allclose(V @ D @ V.T, np.diag(pc.time_eigs(nt, l)), atol=1e-12)
    # eigenvalues against an independent dense eigen-solver
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(D)), np.sort(pc.time_eigs(nt, l)),
                               atol=1e-12)


@pytest.mark.parametrize("nt", [3, 8, 31])
def test_dst1_matches_library(nt):
    V = pc.time_transform(nt, 2)
    ref = sfft.dst(np.eye(nt), type=1, norm="ortho", axis=0)
    np.testing.assert_allclose(V, ref, atol=1e-14)


@pytest.mark.parametrize("bc", ["periodic", "neumann"])
@pytest.mark.parametrize("l", [1, 2])
def test_prec_forms_agree(bc, l):
    g = Grid(d=2, nx=5, ny=4, nt=4, bc=bc, nu=0.3, l=l)
    S = ops.Spatial(g)
    P1 = pc.assemble_P_from_A(g, S)
    P2 = pc.assemble_P_kron(g, S)
    assert abs(P1 - P2).max() <= 1e-13 * abs(P1).max()


@pytest.mark.parametrize("bc", ["periodic", "neumann"])
@pytest.mark.parametrize("l", [1, 2])
@pytest.mark.parametrize("shape", [(1, 9, 1, 5), (2, 6, 5, 4), (2, 8, 8, 7)])
def test_recursive_Pinv_equals_direct(bc, l, shape):
    d, nx, ny, nt = shape
    g = Grid(d=d, nx=nx, ny=ny, nt=nt, bc=bc, nu=0.05, l=l)
    r = np.random.default_rng(5).standard_normal(g.n)
    x_dense = pc.apply_Pinv_dense(g, r)
    x_fast = pc.apply_Pinv_fast(g, r)
    np.testing.assert_allclose(x_fast, x_dense, rtol=0, atol=1e-11 * np.abs(x_dense).max())


@pytest.mark.parametrize("bc", ["periodic", "neumann"])
@pytest.mark.parametrize("l", [1, 2])
@pytest.mark.parametrize("nu", [1.0, 0.01])
def test_lemma1_spectrum(bc, l, nu):
    g = Grid(d=2, nx=4, ny=4, nt=5, bc=bc, nu=nu, l=l)
    S = ops.Spatial(g)
    A = ops.assemble_AAt_blocks(g, S).toarray()
    P = pc.assemble_P_from_A(g, S).toarray()
    ev = np.linalg.eigvals(np.linalg.solve(P, A))
    assert np.abs(ev.imag).max() < 1e-8
    ev = ev.real
    ones = np.sum(np.abs(ev - 1.0) < 1e-8)
    assert ones >= (g.nt - 1) * g.M
    if l == 1:
        assert ev.min() >= 1.0 - 1e-9
    else:
        assert ev.min() > 0 and ev.max() <= 1.0 + 1e-9


@pytest.mark.parametrize("bc", ["periodic", "neumann"])
def test_zero_viscosity_l1_is_exact(bc):
    g = Grid(d=2, nx=6, ny=6, nt=6, bc=bc, nu=0.0, l=1)
    S = ops.Spatial(g)
    A = ops.assemble_AAt_blocks(g, S)
    P = pc.assemble_P_from_A(g, S)
    assert abs(A - P).max() <= 1e-13 * abs(A).max()
    b = np.random.default_rng(2).standard_normal(g.n)
    x, its, rel = cgmod.pcg(lambda v: ops.apply_AAt(g, S, v), lambda r: pc.apply_Pinv_fast(g, r),
                            b, 1e-10, 50)
    assert its == 1
    assert np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b)
