"""Parallel-in-time preconditioner of Section 4.

eq. Adecom writes the reduced matrix with C-hat = nu^2 K^2 + B B^T,
H = (2 nu K + I/dt)/dt and L-hat = L/dt; eq. prec replaces H in the first
diagonal block by l L-hat (l in {1, 2}). Then (Section 4.1)
    P = I_{N_t} (x) C-hat + D_tt (x) L-hat,
with D_tt the tridiagonal (-1, 2, -1) whose first diagonal entry is l, and
D_tt = V^{-1} Lambda_t V with V the DCT-VIII (l = 1) or DST-I (l = 2) and
lambda_k = 2 - 2 cos(pi (k - 1 + l/2) / (N_t + l/2)) (eq. eigs).

Algorithm 1 applies P^{-1} by transforming along time, solving the N_t
independent systems (C-hat + lambda_k L-hat) x_k = y_k (eq. paral) and
transforming back. Section 4.3 shows B B^T = 2K (eq. precstead) and solves
each system exactly by diagonalising K with the DFT (periodic) or the DCT-II
(Neumann), Algorithm 2 / eq. paralrec, which together give eq. pstrec.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .grid import Grid
from .operators import Spatial, assemble_AAt_blocks


def time_eigs(nt: int, l: int) -> np.ndarray:
    """lambda_k, k = 1..N_t (eq. eigs)."""
    k = np.arange(1, nt + 1)
    return 2.0 - 2.0 * np.cos(np.pi * (k - 1 + l / 2.0) / (nt + l / 2.0))


def Dtt(nt: int, l: int) -> np.ndarray:
    """Negative second-difference matrix in time with D_tt[0, 0] = l."""
    D = 2.0 * np.eye(nt) - np.eye(nt, k=1) - np.eye(nt, k=-1)
    D[0, 0] = float(l)
    return D


def time_transform(nt: int, l: int) -> np.ndarray:
    """Orthonormal transform V with V D_tt V^T = diag(lambda_k).

    l = 1: DCT-VIII, V[k, j] = sqrt(4/(2N+1)) cos(pi (2k-1)(2j-1) / (2(2N+1)));
    l = 2: DST-I,    V[k, j] = sqrt(2/(N+1)) sin(pi k j / (N+1)),  k, j = 1..N.
    Both are symmetric, so V^{-1} = V^T = V.
    """
    k = np.arange(1, nt + 1)[:, None]
    j = np.arange(1, nt + 1)[None, :]
    if l == 1:
        return np.sqrt(4.0 / (2 * nt + 1)) * np.cos(
            np.pi * (2 * k - 1) * (2 * j - 1) / (2.0 * (2 * nt + 1)))
    if l == 2:
        return np.sqrt(2.0 / (nt + 1)) * np.sin(np.pi * k * j / (nt + 1.0))
    raise ValueError("l must be 1 or 2")


def laplacian_eigs(N: int, bc: str) -> np.ndarray:
    """Eigenvalues of the unscaled one-axis negative Laplacian (Algorithm 2):
    2 - 2 cos(2 pi v / N) (periodic) or 2 - 2 cos(pi v / N) (Neumann)."""
    v = np.arange(N)
    if bc == "periodic":
        return 2.0 - 2.0 * np.cos(2.0 * np.pi * v / N)
    return 2.0 - 2.0 * np.cos(np.pi * v / N)


def assemble_P_from_A(g: Grid, S: Spatial | None = None):
    """eq. prec as a modification of eq. Adecom: A with the first diagonal
    block's H replaced by l L-hat."""
    S = S or Spatial(g)
    A = assemble_AAt_blocks(g, S)
    H = (2.0 * g.nu * S.K + S.I / g.dt) / g.dt
    Lhat = S.L / g.dt
    e0 = sp.csr_matrix(([1.0], ([0], [0])), shape=(g.nt, g.nt))
    return (A - sp.kron(e0, H - g.l * Lhat)).tocsr()


def assemble_P_kron(g: Grid, S: Spatial | None = None):
    """Kronecker form I (x) C-hat + D_tt (x) L-hat with C-hat = nu^2 K^2 + B B^T."""
    S = S or Spatial(g)
    Chat = g.nu ** 2 * (S.K @ S.K) + S.BBt
    Lhat = S.L / g.dt
    return (sp.kron(sp.identity(g.nt), Chat) + sp.kron(sp.csr_matrix(Dtt(g.nt, g.l)), Lhat)).tocsr()


def apply_Pinv_dense(g: Grid, r: np.ndarray, S: Spatial | None = None) -> np.ndarray:
    """Exact P^{-1} r by a sparse direct solve (small grids only)."""
    P = assemble_P_from_A(g, S)
    return spla.spsolve(P.tocsc(), r)


def spatial_solve(g: Grid, y: np.ndarray, lam: float) -> np.ndarray:
    """Algorithm 2: (C-hat + lambda L-hat)^{-1} y for one time slice.

    R = lambda_x/dx^2 + lambda_y/dy^2 (tiled), S = nu^2 R*R + 2R + (nu lambda/dt) R
    + lambda/dt^2; transform along y then x, divide entrywise by S, invert.
    Each axis takes the transform of its boundary type: the DFT (periodic) or
    the orthonormal DCT-II (Neumann).
    """
    bx, by = g.bcs
    lx = laplacian_eigs(g.nx, bx) / g.dx ** 2
    if g.d == 1:
        R = lx
        Y = y
        axes = ((0, bx),)
    else:
        ly = laplacian_eigs(g.ny, by) / g.dy ** 2
        R = lx[:, None] + ly[None, :]
        Y = y.reshape(g.nx, g.ny)
        axes = ((1, by), (0, bx))
    S = g.nu ** 2 * R * R + 2.0 * R + (g.nu * lam / g.dt) * R + lam / g.dt ** 2
    Yh = Y
    for ax, bc in axes:
        Yh = sfft.fft(Yh, axis=ax) if bc == "periodic" else \
            sfft.dct(Yh, type=2, norm="ortho", axis=ax)
    Xh = Yh / S
    for ax, bc in reversed(axes):
        Xh = sfft.ifft(Xh, axis=ax) if bc == "periodic" else \
            sfft.idct(Xh, type=2, norm="ortho", axis=ax)
    # the result is real (complex only through a DFT axis)
    X = np.real(Xh)
    return np.asarray(X).reshape(-1)


def apply_Pinv_fast(g: Grid, r: np.ndarray) -> np.ndarray:
    """Algorithm 1 with Algorithm 2 as the per-step solver (eq. pstrec)."""
    V = time_transform(g.nt, g.l)
    lam = time_eigs(g.nt, g.l)
    Y = V @ r.reshape(g.nt, g.M)
    X = np.empty_like(Y)
    for k in range(g.nt):
        X[k] = spatial_solve(g, Y[k], lam[k])
    return (V.T @ X).reshape(-1)
