"""Sparse FP64 operators of the discrete variational problem.

Conventions (the paper eliminates m^0 and keeps 5 N_t N_x N_y unknowns,
Section 2.1): the primal vector is y = (m, w^(0), ..., w^(2d-1)); each block
has N_t time slices of M = N_x N_y values in [i][j] order (j fastest). Slice t
of m holds m^{t+1}; slice t of w holds w^t, so that the cost pairs
(m^{t+1}, w^t), as in the scheme (MFG_T^2_h) where the coupling is evaluated
at m^{k+1} and the flux is Phi(u^k) m^{k+1}.

Row t of the reduced constraint (eq. ABC with the first block row removed) is
the discrete Fokker-Planck equation of the constraint map G in (VMFG_h):
    (m^{t+1} - m^t)/dt - nu Lap_h m^{t+1} + div_h w^t = 0,  m^0 = m_0,
i.e.  L m_t - [t >= 1] m_{t-1}/dt + B w_t = [t == 0] m_0 / dt,
with L = nu K + I/dt (Section 3) and K the negative discrete Laplacian.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .grid import Grid


def divergence_factors(N: int, bc: str):
    """D^1, D^2 of Section 4.3 (N x N, unscaled).

    Periodic: D^1 has 1 on the diagonal and -1 below it, with the wrap entry
    D^1[0, N-1] = -1; D^2 = -(D^1)^T.
    Neumann: D^1 = diag(1, ..., 1, 0) with -1 below the diagonal;
    D^2 = diag(0, -1, ..., -1) with 1 above the diagonal.
    """
    if bc == "periodic":
        D1 = sp.lil_matrix((N, N))
        for i in range(N):
            D1[i, i] = 1.0
            D1[i, (i - 1) % N] = -1.0
        D1 = D1.tocsr()
        D2 = (-D1.T).tocsr()
        return D1, D2
    D1 = sp.lil_matrix((N, N))
    D2 = sp.lil_matrix((N, N))
    for i in range(N):
        if i <= N - 2:
            D1[i, i] = 1.0
            D2[i, i + 1] = 1.0
        if i >= 1:
            D1[i, i - 1] = -1.0
            D2[i, i] = -1.0
    return D1.tocsr(), D2.tocsr()


def neg_laplacian_1d(N: int, bc: str, h: float):
    """One-axis negative Laplacian.

    Periodic: (2 u_i - u_{i+1} - u_{i-1}) / h^2 with indices mod N (the
    Section 2 definition of Lap_h). Neumann: the Section 4.3 matrix, the
    tridiagonal (-1, 2, -1) with both corner entries equal to 1, over h^2.
    """
    K = sp.lil_matrix((N, N))
    for i in range(N):
        if bc == "periodic":
            K[i, i] += 2.0
            K[i, (i + 1) % N] += -1.0
            K[i, (i - 1) % N] += -1.0
        else:
            K[i, i] = 2.0 if 0 < i < N - 1 else 1.0
            if i + 1 < N:
                K[i, i + 1] = -1.0
            if i - 1 >= 0:
                K[i, i - 1] = -1.0
    return (K.tocsr() / (h * h)).tocsr()


class Spatial:
    """Per-time-slice spatial matrices (M x M): K, L, the 2d blocks of B, C."""

    def __init__(self, g: Grid):
        self.g = g
        bx, by = g.bcs
        Kx = neg_laplacian_1d(g.nx, bx, g.dx)
        D1x, D2x = divergence_factors(g.nx, bx)
        if g.d == 1:
            self.K = Kx
            self.B = [D1x / g.dx, D2x / g.dx]
        else:
            Ky = neg_laplacian_1d(g.ny, by, g.dy)
            D1y, D2y = divergence_factors(g.ny, by)
            Ix = sp.identity(g.nx, format="csr")
            Iy = sp.identity(g.ny, format="csr")
            self.K = (sp.kron(Kx, Iy) + sp.kron(Ix, Ky)).tocsr()
            self.B = [sp.kron(D1x, Iy).tocsr() / g.dx, sp.kron(D2x, Iy).tocsr() / g.dx,
                      sp.kron(Ix, D1y).tocsr() / g.dy, sp.kron(Ix, D2y).tocsr() / g.dy]
        self.B = [b.tocsr() for b in self.B]
        I = sp.identity(g.M, format="csr")
        self.I = I
        self.L = (g.nu * self.K + I / g.dt).tocsr()
        BBt = sum(b @ b.T for b in self.B)
        self.BBt = BBt.tocsr()
        # C = L^2 + B B^T (Section 3, below eq. largeA)
        self.C = (self.L @ self.L + self.BBt).tocsr()


def assemble_Cr(g: Grid, S: Spatial | None = None):
    """Reduced constraint matrix Cr = [A' | I (x) B] of size n x (1+2d) n."""
    S = S or Spatial(g)
    It = sp.identity(g.nt, format="csr")
    sub = sp.diags([np.ones(g.nt - 1)], [-1], shape=(g.nt, g.nt), format="csr")
    Ap = sp.kron(It, S.L) - sp.kron(sub, S.I / g.dt)
    blocks = [Ap] + [sp.kron(It, b) for b in S.B]
    return sp.hstack(blocks).tocsr()


def rhs_d(g: Grid, m0: np.ndarray) -> np.ndarray:
    """Right-hand side dr of the reduced constraint: m_0/dt in slice 0."""
    d = np.zeros(g.n)
    d[: g.M] = m0 / g.dt
    return d


def assemble_AAt_blocks(g: Grid, S: Spatial | None = None):
    """The reduced system of eq. largeA assembled from its blocks:
    diagonal C (t = 0) and C + I/dt^2 (t >= 1), off-diagonal -L/dt."""
    S = S or Spatial(g)
    nt = g.nt
    diag_sel = sp.diags([np.r_[0.0, np.ones(nt - 1)]], [0], shape=(nt, nt))
    off = sp.diags([np.ones(nt - 1), np.ones(nt - 1)], [-1, 1], shape=(nt, nt))
    A = (sp.kron(sp.identity(nt), S.C) + sp.kron(diag_sel, S.I / g.dt ** 2)
         - sp.kron(off, S.L / g.dt))
    return A.tocsr()


# ---------------------------------------------------------------------------
# Slice-wise application (any size): the same block structure as above, applied
# one time slice at a time with the M x M spatial matrices.
# ---------------------------------------------------------------------------

def apply_AAt(g: Grid, S: Spatial, u: np.ndarray) -> np.ndarray:
    """(A u)_t = C u_t + [t>=1] u_t/dt^2 - L (u_{t-1} + u_{t+1})/dt (eq. largeA)."""
    U = u.reshape(g.nt, g.M)
    Q = np.empty_like(U)
    for t in range(g.nt):
        q = S.C @ U[t]
        if t >= 1:
            q += U[t] / g.dt ** 2
        nb = np.zeros(g.M)
        if t >= 1:
            nb += U[t - 1]
        if t <= g.nt - 2:
            nb += U[t + 1]
        q -= (S.L @ nb) / g.dt
        Q[t] = q
    return Q.reshape(-1)


def apply_Cr(g: Grid, S: Spatial, y: np.ndarray) -> np.ndarray:
    """Cr y, slice by slice: L m_t - [t>=1] m_{t-1}/dt + sum_c B_c w^(c)_t."""
    nb = 1 + g.ncomp
    Y = y.reshape(nb, g.nt, g.M)
    out = np.empty((g.nt, g.M))
    for t in range(g.nt):
        r = S.L @ Y[0, t]
        if t >= 1:
            r -= Y[0, t - 1] / g.dt
        for c in range(g.ncomp):
            r += S.B[c] @ Y[1 + c, t]
        out[t] = r
    return out.reshape(-1)


def apply_CrT(g: Grid, S: Spatial, u: np.ndarray) -> np.ndarray:
    """Cr^T u, slice by slice: m-part L u_t - [t<=N_t-2] u_{t+1}/dt,
    w-parts B_c^T u_t."""
    U = u.reshape(g.nt, g.M)
    out = np.empty((1 + g.ncomp, g.nt, g.M))
    for t in range(g.nt):
        r = S.L @ U[t]
        if t <= g.nt - 2:
            r -= U[t + 1] / g.dt
        out[0, t] = r
        for c in range(g.ncomp):
            out[1 + c, t] = S.B[c].T @ U[t]
    return out.reshape(-1)


def abs_AAt_bound(g: Grid, S: Spatial, u: np.ndarray) -> np.ndarray:
    """|A| |u| entrywise, built from the absolute spatial blocks |C| and |L|;
    the scale against which a rounding error of an A-product is measured."""
    Ca = abs(S.C)
    La = abs(S.L)
    U = np.abs(u.reshape(g.nt, g.M))
    Q = np.empty_like(U)
    for t in range(g.nt):
        q = Ca @ U[t]
        if t >= 1:
            q += U[t] / g.dt ** 2
        nb = np.zeros(g.M)
        if t >= 1:
            nb += U[t - 1]
        if t <= g.nt - 2:
            nb += U[t + 1]
        q += (La @ nb) / g.dt
        Q[t] = q
    return Q.reshape(-1)


def abs_Cr_bound(g: Grid, S: Spatial, y: np.ndarray) -> np.ndarray:
    """|Cr| |y| entrywise (slice-wise)."""
    La = abs(S.L)
    Ba = [abs(b) for b in S.B]
    nb = 1 + g.ncomp
    Y = np.abs(y.reshape(nb, g.nt, g.M))
    out = np.empty((g.nt, g.M))
    for t in range(g.nt):
        r = La @ Y[0, t]
        if t >= 1:
            r += Y[0, t - 1] / g.dt
        for c in range(g.ncomp):
            r += Ba[c] @ Y[1 + c, t]
        out[t] = r
    return out.reshape(-1)


def abs_CrT_bound(g: Grid, S: Spatial, u: np.ndarray) -> np.ndarray:
    """|Cr^T| |u| entrywise (slice-wise)."""
    La = abs(S.L)
    Ba = [abs(b) for b in S.B]
    U = np.abs(u.reshape(g.nt, g.M))
    out = np.empty((1 + g.ncomp, g.nt, g.M))
    for t in range(g.nt):
        r = La @ U[t]
        if t <= g.nt - 2:
            r += U[t + 1] / g.dt
        out[0, t] = r
        for c in range(g.ncomp):
            out[1 + c, t] = Ba[c].T @ U[t]
    return out.reshape(-1)
