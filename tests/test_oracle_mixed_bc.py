"""Pins of the oracle with a boundary type per axis (d = 2; Section 4.3 notes
that the spatial solver allows different conditions in x and y).

* The mixed negative Laplacian has the separable eigenvectors fixed by each
  axis's type: cos(pi p (i + 1/2)/N_x) on a Neumann x axis (eigenvalue
  (2 - 2cos(pi p/N_x))/dx^2) times cos / sin(2 pi q j/N_y) on a periodic y axis
  ((2 - 2cos(2 pi q/N_y))/dy^2), and the same with the axes exchanged.
* B B^T = 2K (eq. precstead holds axis by axis), and every column of K and of
  the divergence blocks sums to zero (the scheme conserves mass).
* eq. prec assembled from A equals its Kronecker form; Algorithms 1 + 2 with a
  DFT on the periodic axis and a DCT-II on the Neumann axis reproduce a sparse
  direct solve with the assembled P; Lemma 1's spectrum statements hold.
* A pair of equal types is the single-type grid.
* The uniform density (V = 0, m0 = 1) is an equilibrium of the CP iteration.
"""
import numpy as np
import pytest

from oracle import cp as ocp
from oracle import operators as ops
from oracle import precond as pc
from oracle.grid import Grid

MIXED = [("neumann", "periodic"), ("periodic", "neumann")]


def _eigvec_1d(N, bc, k):
    """Closed-form eigenvectors of the one-axis negative Laplacian for mode k
    (two for a periodic mode 0 < k < N/2: cosine and sine)."""
    i = np.arange(N)
    if bc == "neumann":
        return [np.cos(np.pi * k * (i + 0.5) / N)], (2 - 2 * np.cos(np.pi * k / N))
    vs = [np.cos(2 * np.pi * k * i / N)]
    if 0 < k and 2 * k != N:
        vs.append(np.sin(2 * np.pi * k * i / N))
    return vs, (2 - 2 * np.cos(2 * np.pi * k / N))


@pytest.mark.parametrize("bcs", MIXED)
@pytest.mark.parametrize("shape", [(6, 5), (8, 9)])
def test_mixed_laplacian_separable_eigenvectors(bcs, shape):
    nx, ny = shape
    g = Grid(d=2, nx=nx, ny=ny, nt=3, bc=bcs, nu=0.2, lo=(0.0, -0.5), hi=(1.0, 0.7))
    # spacing of each axis from its own type
    assert g.dx == pytest.approx(1.0 / (nx + (bcs[0] == "neumann")))
    assert g.dy == pytest.approx(1.2 / (ny + (bcs[1] == "neumann")))
    K = ops.Spatial(g).K
    for p in range(nx):
        vx, lx = _eigvec_1d(nx, bcs[0], p)
        for q in range(ny):
            vy, ly = _eigvec_1d(ny, bcs[1], q)
            lam = lx / g.dx ** 2 + ly / g.dy ** 2
            for a in vx:
                for b in vy:
                    v = np.outer(a, b).reshape(-1)
                    np.testing.assert_allclose(K @ v, lam * v, rtol=0,
                                               atol=1e-12 * (1 + lam) * np.abs(v).max())


@pytest.mark.parametrize("bcs", MIXED)
def test_mixed_BBt_and_mass(bcs):
    g = Grid(d=2, nx=6, ny=5, nt=3, bc=bcs, nu=0.2)
    S = ops.Spatial(g)
    assert abs(S.BBt - 2 * S.K).max() <= 1e-14 * abs(S.K).max()
    ones = np.ones(g.M)
    assert np.abs(ones @ S.K).max() <= 1e-12 * abs(S.K).max()
    for b in S.B:
        assert np.abs(ones @ b).max() <= 1e-12 * abs(b).max()
    # the Neumann axis has structurally zero divergence columns, the periodic none
    nz = [np.asarray(abs(b).sum(axis=0)).ravel() == 0 for b in S.B]
    x_neu, y_neu = (bc == "neumann" for bc in bcs)
    assert nz[0].any() == x_neu and nz[1].any() == x_neu
    assert nz[2].any() == y_neu and nz[3].any() == y_neu


@pytest.mark.parametrize("bcs", MIXED)
@pytest.mark.parametrize("l", [1, 2])
def test_mixed_prec_forms_agree(bcs, l):
    g = Grid(d=2, nx=5, ny=4, nt=4, bc=bcs, nu=0.3, l=l)
    S = ops.Spatial(g)
    P1 = pc.assemble_P_from_A(g, S)
    P2 = pc.assemble_P_kron(g, S)
    assert abs(P1 - P2).max() <= 1e-13 * abs(P1).max()


@pytest.mark.parametrize("bcs", MIXED)
@pytest.mark.parametrize("l", [1, 2])
@pytest.mark.parametrize("shape", [(6, 5, 4), (8, 9, 7)])
def test_mixed_recursive_Pinv_equals_direct(bcs, l, shape):
    nx, ny, nt = shape
    g = Grid(d=2, nx=nx, ny=ny, nt=nt, bc=bcs, nu=0.05, l=l)
    r = np.random.default_rng(7).standard_normal(g.n)
    x_dense = pc.apply_Pinv_dense(g, r)
    x_fast = pc.apply_Pinv_fast(g, r)
    np.testing.assert_allclose(x_fast, x_dense, rtol=0, atol=1e-11 * np.abs(x_dense).max())


@pytest.mark.parametrize("bcs", MIXED)
@pytest.mark.parametrize("l", [1, 2])
def test_mixed_lemma1_spectrum(bcs, l):
    g = Grid(d=2, nx=4, ny=5, nt=5, bc=bcs, nu=0.3, l=l)
    S = ops.Spatial(g)
    A = ops.assemble_AAt_blocks(g, S).toarray()
    P = pc.assemble_P_from_A(g, S).toarray()
    ev = np.linalg.eigvals(np.linalg.solve(P, A))
    assert np.abs(ev.imag).max() < 1e-8
    ev = ev.real
    assert np.sum(np.abs(ev - 1.0) < 1e-8) >= (g.nt - 1) * g.M
    if l == 1:
        assert ev.min() >= 1.0 - 1e-9
    else:
        assert ev.min() > 0 and ev.max() <= 1.0 + 1e-9


@pytest.mark.parametrize("bc", ["periodic", "neumann"])
def test_equal_pair_is_single_type(bc):
    a = Grid(d=2, nx=5, ny=6, nt=4, bc=bc, nu=0.1)
    b = Grid(d=2, nx=5, ny=6, nt=4, bc=(bc, bc), nu=0.1)
    assert (a.dx, a.dy) == (b.dx, b.dy)
    Sa, Sb = ops.Spatial(a), ops.Spatial(b)
    assert abs(Sa.K - Sb.K).max() == 0
    r = np.random.default_rng(1).standard_normal(a.n)
    assert np.array_equal(pc.apply_Pinv_fast(a, r), pc.apply_Pinv_fast(b, r))


def test_per_axis_bc_needs_two_dimensions():
    with pytest.raises(ValueError):
        Grid(d=1, nx=5, ny=1, nt=3, bc=("periodic", "neumann"), nu=0.1)
    with pytest.raises(ValueError):
        Grid(d=2, nx=5, ny=5, nt=3, bc=("periodic", "dirichlet"), nu=0.1)


@pytest.mark.parametrize("bcs", MIXED)
def test_mixed_uniform_equilibrium(bcs):
    g = Grid(d=2, nx=6, ny=5, nt=6, bc=bcs, nu=0.1)
    m0 = np.ones(g.M)
    st, _ = ocp.cp_solve(g, np.zeros(g.M), m0, 150, method="direct")
    np.testing.assert_allclose(st.y[: g.n], 1.0, atol=1e-6)
    assert np.abs(st.y[g.n:]).max() <= 1e-6
