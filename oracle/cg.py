"""Conjugate gradients on the reduced SPD system (Sections 3-4).

The reduced matrix of eq. largeA is symmetric positive definite, so the
projection of each Chambolle-Pock step is a CG solve. The paper runs SciPy's
CG: zero initial guess, stop when the recursively updated residual satisfies
||r||_2 <= rtol ||b||_2. Both the plain method and the preconditioned one
(with the Section 4 preconditioner applied as an SPD operator) are given,
plus the flexible variant (Polak-Ribiere beta) used when the preconditioner
is applied inexactly.
"""
from __future__ import annotations

import numpy as np


def cg(apply_A, b: np.ndarray, rtol: float, maxit: int, x0=None):
    """Unpreconditioned CG. Returns (x, iters, relres_recursive)."""
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - apply_A(x) if x0 is not None else b.copy()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros_like(b), 0, 0.0
    p = r.copy()
    rr = float(r @ r)
    it = 0
    while np.sqrt(rr) > rtol * bnorm and it < maxit:
        q = apply_A(p)
        alpha = rr / float(p @ q)
        x += alpha * p
        r -= alpha * q
        rr_new = float(r @ r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return x, it, np.sqrt(rr) / bnorm


def pcg(apply_A, apply_Pinv, b: np.ndarray, rtol: float, maxit: int,
        flexible: bool = False, x0=None):
    """Preconditioned CG from x0 (default 0). Returns (x, iters, relres_recursive).
    The stopping rule is ||r|| <= rtol ||b|| whatever the start.

    Standard: beta = (r'.z')/(r.z). Flexible: beta = z'.(r' - r)/(r.z),
    evaluated as -alpha (z'.q)/(r.z) since r' - r = -alpha q.
    """
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros_like(b), 0, 0.0
    r = b.copy() if x0 is None else b - apply_A(x)
    z = apply_Pinv(r)
    p = z.copy()
    rho = float(r @ z)
    it = 0
    rn = bnorm
    while it < maxit:
        q = apply_A(p)
        alpha = rho / float(p @ q) if rho != 0.0 else 0.0
        x += alpha * p
        r -= alpha * q
        it += 1
        rn = np.linalg.norm(r)
        if rn <= rtol * bnorm:
            break
        z = apply_Pinv(r)
        rho_new = float(r @ z)
        if flexible:
            beta = -alpha * float(z @ q) / rho
        else:
            beta = rho_new / rho
        p = z + beta * p
        rho = rho_new
    return x, it, rn / bnorm
