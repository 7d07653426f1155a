"""Pins of the oracle against the matrices the paper prints (Section 4).

The fixture `golden/section4_matrices_n5.txt` holds those matrices written out
by hand at size 5: D_tt for l = 1, 2 (Section 4.2), the periodic and Neumann
divergence factors D^1_x, D^2_x and their products with their transposes
(Section 4.3). The tests compare the oracle's builders with them entry by
entry, and check the statements the paper makes about them: D D^T of either
factor gives the printed product, B B^T = 2/dx^2 times it, and the printed D_tt
has the eigenvalues of eq. eigs and is diagonalised by the transform V.
"""
import pathlib

import numpy as np
import pytest

from oracle import operators as ops
from oracle import precond as pc
from oracle.grid import Grid

FIXTURE = pathlib.Path(__file__).parent / "golden" / "section4_matrices_n5.txt"


def _load_blocks(path):
    blocks, name, rows = {}, None, []
    for line in path.read_text().splitlines():
        s = line.strip()
        if s.startswith("## "):
            if name is not None:
                blocks[name] = np.array(rows, dtype=np.float64)
            name, rows = s[3:].strip(), []
        elif s and not s.startswith("#"):
            rows.append([float(v) for v in s.split()])
    if name is not None:
        blocks[name] = np.array(rows, dtype=np.float64)
    return blocks


G = _load_blocks(FIXTURE)


def test_fixture_is_complete():
    names = {"Dtt_l1", "Dtt_l2", "D1_periodic", "D2_periodic", "D1_neumann",
             "D2_neumann", "DDt_periodic", "DDt_neumann"}
    assert set(G) == names
    assert all(G[k].shape == (5, 5) for k in names)


@pytest.mark.parametrize("bc", ["periodic", "neumann"])
def test_divergence_factors_match_printed(bc):
    D1, D2 = ops.divergence_factors(5, bc)
    np.testing.assert_array_equal(D1.toarray(), G[f"D1_{bc}"])
    np.testing.assert_array_equal(D2.toarray(), G[f"D2_{bc}"])


@pytest.mark.parametrize("bc", ["periodic", "neumann"])
def test_printed_products_are_consistent(bc):
    # the paper states that both factors give the same product with their transposes
    D1, D2, DDt = G[f"D1_{bc}"], G[f"D2_{bc}"], G[f"DDt_{bc}"]
    np.testing.assert_array_equal(D1 @ D1.T, DDt)
    np.testing.assert_array_equal(D2 @ D2.T, DDt)


@pytest.mark.parametrize("bc", ["periodic", "neumann"])
def test_laplacian_matches_printed(bc):
    K = ops.neg_laplacian_1d(5, bc, 1.0).toarray()
    np.testing.assert_array_equal(K, G[f"DDt_{bc}"])


@pytest.mark.parametrize("bc", ["periodic", "neumann"])
def test_BBt_matches_printed(bc):
    g = Grid(d=1, nx=5, ny=1, nt=3, bc=bc, nu=0.1)
    S = ops.Spatial(g)
    # dx = 1/5 for the torus, 1/6 for the Neumann interior grid (Section 4.3)
    assert g.dx == pytest.approx(1 / 5 if bc == "periodic" else 1 / 6, rel=1e-15)
    ref = 2.0 / g.dx ** 2 * G[f"DDt_{bc}"]
    np.testing.assert_allclose(S.BBt.toarray(), ref, rtol=1e-14, atol=0)


@pytest.mark.parametrize("l", [1, 2])
def test_Dtt_matches_printed(l):
    np.testing.assert_array_equal(pc.Dtt(5, l), G[f"Dtt_l{l}"])


@pytest.mark.parametrize("l", [1, 2])
def test_printed_Dtt_spectrum_and_transform(l):
    D = G[f"Dtt_l{l}"]
    lam = pc.time_eigs(5, l)
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(D)), np.sort(lam), atol=1e-13)
    V = pc.time_transform(5, l)
    np.testing.assert_allclose(V @ D @ V.T, np.diag(lam), atol=1e-13)
