"""Pins of the oracle's conjugate-gradient variants (Sections 3-4).

* Plain CG solves an SPD system to its stopping rule and its iterates match a
  dense solve.
* Flexible PCG (beta = z'.(r' - r)/(r.z)) with an exact SPD preconditioner
  produces the same iterates as standard PCG up to rounding, because the
  residuals are then P^{-1}-conjugate and z'.r = 0; with the identity
  preconditioner it is plain CG.
* With a slightly non-symmetric preconditioner (the situation of a
  low-precision preconditioner) flexible PCG still converges to the tolerance.
"""
import numpy as np

from oracle import cg


def _spd(n, cond, rng):
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.logspace(0, np.log10(cond), n)
    return (Q * ev) @ Q.T


def test_plain_cg_matches_dense_solve():
    rng = np.random.default_rng(1)
    A = _spd(60, 1e4, rng)
    b = rng.standard_normal(60)
    x, it, rel = cg.cg(lambda v: A @ v, b, 1e-12, 1000)
    assert rel <= 1e-12
    assert np.linalg.norm(A @ x - b) <= 1.01e-12 * np.linalg.norm(b)
    xs = np.linalg.solve(A, b)
    assert np.abs(x - xs).max() <= 1e-7 * np.abs(xs).max()


def test_flexible_equals_standard_with_exact_preconditioner():
    rng = np.random.default_rng(2)
    A = _spd(80, 1e5, rng)
    P = A + _spd(80, 10, rng) * 0.3          # SPD preconditioner close to A
    Pinv = np.linalg.inv(P)
    b = rng.standard_normal(80)
    for k in [1, 3, 6, 10]:         # the k-th iterates (no stopping test: rtol = 0)
        xs, its_s, rs = cg.pcg(lambda v: A @ v, lambda r: Pinv @ r, b, 0.0, k)
        xf, its_f, rf = cg.pcg(lambda v: A @ v, lambda r: Pinv @ r, b, 0.0, k, flexible=True)
        assert its_s == its_f == k
        assert np.abs(xs - xf).max() <= 1e-10 * np.abs(xs).max()
        assert abs(rs - rf) <= 1e-8 * rs


def test_flexible_with_identity_is_plain_cg():
    rng = np.random.default_rng(3)
    A = _spd(200, 30.0, rng)
    b = rng.standard_normal(200)
    for k in [1, 5, 12, 25]:        # the k-th iterates (no stopping test: rtol = 0)
        x0, it0, _ = cg.cg(lambda v: A @ v, b, 0.0, k)
        x1, it1, _ = cg.pcg(lambda v: A @ v, lambda r: r.copy(), b, 0.0, k, flexible=True)
        assert it0 == it1 == k
        assert np.abs(x0 - x1).max() <= 1e-12 * np.abs(x0).max()


def test_flexible_converges_with_perturbed_preconditioner():
    rng = np.random.default_rng(4)
    A = _spd(120, 1e6, rng)
    Pinv = np.linalg.inv(A + _spd(120, 10, rng) * 0.1)
    # relative, non-symmetric error of 1e-3, as a low-precision preconditioner has
    E = rng.standard_normal((120, 120)) * 1e-3 / np.sqrt(120)
    Pe = (np.eye(120) + E) @ Pinv
    b = rng.standard_normal(120)
    x, it, rel = cg.pcg(lambda v: A @ v, lambda r: Pe @ r, b, 1e-10, 400, flexible=True)
    assert rel <= 1e-10
    assert np.linalg.norm(A @ x - b) <= 1e-9 * np.linalg.norm(b)


def test_pcg_warm_start():
    """From x0 the residual is b - A x0 and the stopping rule stays relative to
    ||b||: a start at the (rounded) solution stops after one step; a start near it needs
    fewer iterations than a cold start and reaches the same tolerance."""
    rng = np.random.default_rng(5)
    A = _spd(100, 1e4, rng)
    Pinv = np.linalg.inv(A + _spd(100, 10, rng) * 0.5)
    b = rng.standard_normal(100)
    xs = np.linalg.solve(A, b)
    x, it, rel = cg.pcg(lambda v: A @ v, lambda r: Pinv @ r, b, 1e-8, 200, x0=xs)
    assert it == 1 and np.linalg.norm(A @ x - b) <= 1e-12 * np.linalg.norm(b)
    x_cold, it_cold, _ = cg.pcg(lambda v: A @ v, lambda r: Pinv @ r, b, 1e-10, 200)
    near = xs + 1e-6 * rng.standard_normal(100) * np.abs(xs).max()
    x_warm, it_warm, rel = cg.pcg(lambda v: A @ v, lambda r: Pinv @ r, b, 1e-10, 200, x0=near)
    assert rel <= 1e-10 and it_warm < it_cold
    assert np.linalg.norm(A @ x_warm - b) <= 1.01e-10 * np.linalg.norm(b)
