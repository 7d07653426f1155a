"""Pins of the oracle's discrete operators against what the paper fixes.

* K spectrum: closed forms of Algorithm 2 (2 - 2cos(2 pi v/N), 2 - 2cos(pi v/N)).
* D^1 (D^1)^T = D^2 (D^2)^T = unscaled Laplacian, so B B^T = 2K (eq. precstead).
* Column sums of D^1, D^2, K vanish (mass conservation of the scheme).
* Cr y - dr equals the constraint map G of (VMFG_h) evaluated directly from the
  Section 2 difference operators (periodic torus, index arithmetic mod N).
* Cr Cr^T equals the block matrix of eq. largeA (two independent assemblies).
* Slice-wise products equal the assembled sparse products.
* lambda_min of the reduced matrix equals lambda_1(l=1)/dt^2 (constant-in-space
  vectors reduce it to D_tt(l=1)/dt^2, the smallest part of the spectrum).
"""
import numpy as np
import pytest

from oracle import operators as ops
from oracle import precond as pc
from oracle.grid import Grid


@pytest.mark.parametrize("bc", ["periodic", "neumann"])
@pytest.mark.parametrize("N", [4, 5, 8, 13])
def test_laplacian_spectrum_closed_form(bc, N):
    h = 0.37
    K = ops.neg_laplacian_1d(N, bc, h).toarray()
    ev = np.sort(np.linalg.eigvalsh(K))
    v = np.arange(N)
    closed = (2 - 2 * np.cos((2 if bc == "periodic" else 1) * np.pi * v / N)) / h ** 2
    np.testing.assert_allclose(ev, np.sort(closed), atol=1e-12 / h ** 2)


@pytest.mark.parametrize("bc", ["periodic", "neumann"])
@pytest.mark.parametrize("N", [4, 7, 16])
def test_divergence_factors(bc, N):
    D1, D2 = ops.divergence_factors(N, bc)
    K1 = ops.neg_laplacian_1d(N, bc, 1.0).toarray()
    np.testing.assert_allclose((D1 @ D1.T).toarray(), K1, atol=0)
    np.testing.assert_allclose((D2 @ D2.T).toarray(), K1, atol=0)
    # zero column sums: the divergence conserves mass
    assert np.abs(np.asarray(D1.sum(axis=0))).max() == 0
    assert np.abs(np.asarray(D2.sum(axis=0))).max() == 0
    assert np.abs(K1.sum(axis=0)).max() == 0
    if bc == "neumann":
        # structurally zero columns: w^(1) at the last node, w^(2) at the first
        assert D1[:, N - 1].nnz == 0 and D2[:, 0].nnz == 0


@pytest.mark.parametrize("bc", ["periodic", "neumann"])
@pytest.mark.parametrize("d", [1, 2])
def test_BBt_equals_2K(bc, d):
    g = Grid(d=d, nx=6, ny=5 if d == 2 else 1, nt=3, bc=bc, nu=0.2)
    S = ops.Spatial(g)
    scale = abs(S.K).max()
    assert abs(S.BBt - 2 * S.K).max() <= 1e-14 * scale


def _G_direct_periodic(g, m0, y):
    """Constraint map of (VMFG_h), rows k = 0..N_t-1, from the Section 2
    definitions with periodic index arithmetic (np.roll)."""
    nb = 1 + g.ncomp
    Y = y.reshape(nb, g.nt, g.nx, g.ny)
    m = np.concatenate([m0.reshape(1, g.nx, g.ny), Y[0]], axis=0)  # m^0..m^{N_t}
    out = np.empty((g.nt, g.nx, g.ny))
    for k in range(g.nt):
        mk1 = m[k + 1]
        lap = (np.roll(mk1, -1, 0) - 2 * mk1 + np.roll(mk1, 1, 0)) / g.dx ** 2
        if g.d == 2:
            lap += (np.roll(mk1, -1, 1) - 2 * mk1 + np.roll(mk1, 1, 1)) / g.dy ** 2
        w = Y[1:, k]
        D1 = lambda a: (np.roll(a, -1, 0) - a) / g.dx
        div = np.roll(D1(w[0]), 1, 0) + D1(w[1])
        if g.d == 2:
            D2 = lambda a: (np.roll(a, -1, 1) - a) / g.dy
            div += np.roll(D2(w[2]), 1, 1) + D2(w[3])
        out[k] = (m[k + 1] - m[k]) / g.dt - g.nu * lap + div
    return out.reshape(-1)


@pytest.mark.parametrize("d", [1, 2])
def test_Cr_matches_section2_definition(d):
    g = Grid(d=d, nx=7, ny=6 if d == 2 else 1, nt=4, bc="periodic", nu=0.3)
    rng = np.random.default_rng(11)
    y = rng.standard_normal((1 + g.ncomp) * g.n)
    m0 = rng.standard_normal(g.M)
    Cr = ops.assemble_Cr(g)
    lhs = Cr @ y - ops.rhs_d(g, m0)
    rhs = _G_direct_periodic(g, m0, y)
    np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-11 * np.abs(rhs).max())


@pytest.mark.parametrize("bc", ["periodic", "neumann"])
@pytest.mark.parametrize("d", [1, 2])
def test_CrCrT_equals_block_formula(bc, d):
    g = Grid(d=d, nx=6, ny=5 if d == 2 else 1, nt=5, bc=bc, nu=0.07)
    S = ops.Spatial(g)
    Cr = ops.assemble_Cr(g, S)
    A1 = (Cr @ Cr.T).tocsr()
    A2 = ops.assemble_AAt_blocks(g, S)
    assert abs(A1 - A2).max() <= 1e-13 * abs(A1).max()
    # mass: summing a constraint row over space leaves only the time difference
    ones = np.ones(g.M)
    assert np.abs(ones @ S.K).max() <= 1e-12 * abs(S.K).max()
    for b in S.B:
        assert np.abs(ones @ b).max() <= 1e-12 * abs(b).max()


@pytest.mark.parametrize("bc", ["periodic", "neumann"])
@pytest.mark.parametrize("d", [1, 2])
def test_slicewise_products_equal_assembled(bc, d):
    g = Grid(d=d, nx=5, ny=4 if d == 2 else 1, nt=6, bc=bc, nu=0.5)
    S = ops.Spatial(g)
    Cr = ops.assemble_Cr(g, S)
    rng = np.random.default_rng(3)
    u = rng.standard_normal(g.n)
    y = rng.standard_normal((1 + g.ncomp) * g.n)
    A = ops.assemble_AAt_blocks(g, S)
    for got, ref in [(ops.apply_AAt(g, S, u), A @ u), (ops.apply_Cr(g, S, y), Cr @ y),
                     (ops.apply_CrT(g, S, u), Cr.T @ u)]:
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("bc", ["periodic", "neumann"])
def test_lambda_min_of_reduced_matrix(bc):
    g = Grid(d=2, nx=4, ny=4, nt=5, bc=bc, nu=0.1)
    A = ops.assemble_AAt_blocks(g).toarray()
    lmin = np.linalg.eigvalsh(A)[0]
    expect = pc.time_eigs(g.nt, 1)[0] / g.dt ** 2
    assert abs(lmin - expect) <= 1e-9 * expect
