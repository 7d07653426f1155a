"""Proximal step of phi = B-hat + F, cell by cell (Section 3).

For q' = 2 (so q = 2) the per-cell cost is b-hat(m, w) + F(x, m) with
b-hat(m, w) = |w|^2 / (2 m) for m > 0 and w in the cone
K = [0,inf) x (-inf,0] x [0,inf) x (-inf,0] (one sign pair per axis),
b-hat(0, 0) = 0, +inf otherwise; and F(x, m) = m^2/2 + V(x) m for m >= 0,
the primitive of the coupling f(x, m) = m + V(x).

The paper takes the prox from a corollary of an earlier work that is not
reproduced in it; the steps below are derived from the definition of the
proximal operator (eq. def_prox_operator):

  prox_{tau phi}(mbar, wbar) = argmin  b-hat(m, w) + F(m)
                                       + (|m - mbar|^2 + |w - wbar|^2)/(2 tau).

1. For fixed m > 0 the w-problem separates per component and its minimiser is
   w = m/(m + tau) * P_K(wbar) (P_K clips each component to its sign, Section 2).
2. With a = |P_K(wbar)|^2 the remaining m-problem is
   h(m) = a/(2(m + tau)) + m^2/2 + V m + (m - mbar)^2/(2 tau) + const, m >= 0,
   which is convex with h'(m) = -a/(2(m+tau)^2) + (1 + 1/tau) m + V - mbar/tau.
3. If h'(0) >= 0, i.e. 2 tau^2 V - 2 tau mbar - a >= 0, then m = 0 and w = 0.
4. Otherwise h' is increasing and concave on m >= 0, so Newton's method started
   at the root for a = 0, max(0, (mbar - tau V)/(1 + tau)), which lies left of
   the root, rises monotonically towards it. Iterate while an update still
   increases m (at most 64 updates).
"""
from __future__ import annotations

import numpy as np

MAX_NEWTON = 64


def project_cone(wbar: np.ndarray) -> np.ndarray:
    """P_K applied to an array of shape (2d, ...): even components are clipped
    to [0, inf), odd ones to (-inf, 0]."""
    w = np.array(wbar, dtype=np.float64, copy=True)
    w[0::2] = np.maximum(w[0::2], 0.0)
    w[1::2] = np.minimum(w[1::2], 0.0)
    return w


def prox_cells(mbar: np.ndarray, wbar: np.ndarray, V: np.ndarray, tau: float,
               return_iters: bool = False):
    """Vectorised per-cell prox. mbar, V: shape (N,); wbar: shape (2d, N).
    Returns (m, w) (and the Newton update count per cell if asked)."""
    mbar = np.asarray(mbar, dtype=np.float64)
    V = np.broadcast_to(np.asarray(V, dtype=np.float64), mbar.shape)
    wt = project_cone(wbar)
    a = np.sum(wt * wt, axis=0)
    zero = (2.0 * tau * tau * V - 2.0 * tau * mbar - a) >= 0.0
    m = np.maximum(0.0, (mbar - tau * V) / (1.0 + tau))
    iters = np.zeros(mbar.shape, dtype=np.int64)
    active = ~zero
    for _ in range(MAX_NEWTON):
        if not active.any():
            break
        s = m + tau
        hp = -a / (2.0 * s * s) + (1.0 + 1.0 / tau) * m + V - mbar / tau
        hpp = a / (s * s * s) + 1.0 + 1.0 / tau
        m_new = m - hp / hpp
        up = active & (m_new > m)
        m = np.where(up, m_new, m)
        iters += up
        active = up
    m = np.where(zero, 0.0, m)
    w = (m / (m + tau)) * wt
    w[:, zero] = 0.0
    if return_iters:
        return m, w, iters
    return m, w


def prox_primal(g, y: np.ndarray, V: np.ndarray, tau: float) -> np.ndarray:
    """prox_{tau phi} on a whole primal vector y = (m, w^(0..2d-1)), each block
    of N_t x M values; V (length M) is the same at every time slice."""
    nb = 1 + g.ncomp
    Y = y.reshape(nb, g.nt * g.M)
    Vt = np.tile(V, g.nt)
    m, w = prox_cells(Y[0], Y[1:], Vt, tau)
    return np.concatenate([m[None], w], axis=0).reshape(-1)


def cell_objective(m, w, mbar, wbar, V, tau):
    """Per-cell objective of the prox problem (for checks)."""
    w = np.asarray(w, dtype=np.float64)
    wbar = np.asarray(wbar, dtype=np.float64)
    if m < 0:
        return np.inf
    if np.any(w[0::2] < 0) or np.any(w[1::2] > 0):
        return np.inf
    if m == 0:
        if np.any(w != 0):
            return np.inf
        bh = 0.0
    else:
        bh = float(np.dot(w, w)) / (2.0 * m)
    F = 0.5 * m * m + V * m
    return bh + F + ((m - mbar) ** 2 + float(np.dot(w - wbar, w - wbar))) / (2.0 * tau)
