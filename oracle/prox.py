"""Proximal step of phi = B-hat + F (+ G/dt on the last slice), cell by cell
(Section 3; the costs of Section 2.1 and the two problems of Section 5).

For q' = 2 (so q = 2) the per-cell cost is b-hat(m, w) + F(x, m) with
b-hat(m, w) = |w|^2 / (2 m) for m > 0 and w in the cone
K = [0,inf) x (-inf,0] x [0,inf) x (-inf,0] (one sign pair per axis),
b-hat(0, 0) = 0, +inf otherwise. The coupling is a polynomial in m,
    f(x, m) = c2 m^2 + c1 m + V(x),      c2, c1 >= 0,
so F(x, m) = c2 m^3/3 + c1 m^2/2 + V(x) m for m >= 0 (its primitive, Section
2.1). The default (c2, c1) = (0, 1) is f = m + V. Problem 1 of Section 5.1 is
f = (m^2 - sin 2 pi y - sin 2 pi x - cos 4 pi x)/2, i.e. c2 = 1/2, c1 = 0 and
V = -(sin 2 pi y + sin 2 pi x + cos 4 pi x)/2; Problem 2 of Section 5.2 has
f = 0 (c2 = c1 = 0, V = 0). A terminal cost g(x, m) = (m - mbar_T(x))/beta
(Section 5.2) enters the discrete objective as G(x, m^{N_t})/dt with
G = (m^2/2 - mbar_T m)/beta (the term of the functional F in Section 2.1 that
is weighted by 1/dt), so on the last time slice it adds 1/(beta dt) to c1 and
-mbar_T/(beta dt) to V.

The Hamiltonian |p|^q'/q' of eq. power_hamiltonian makes the flux cost
b-hat(m, w) = |w|^q/(q m^(q-1)) with q = q'/(q' - 1) (Section 2.2); the
default and the paper's experiments take q' = q = 2. General q is handled
after the q = 2 steps below (prox_cells_q).

The paper takes the prox from a corollary of an earlier work that is not
reproduced in it; the steps below are derived from the definition of the
proximal operator (eq. def_prox_operator):

  prox_{tau phi}(mbar, wbar) = argmin  b-hat(m, w) + F(m)
                                       + (|m - mbar|^2 + |w - wbar|^2)/(2 tau).

1. For fixed m > 0 the w-problem separates per component and its minimiser is
   w = m/(m + tau) * P_K(wbar) (P_K clips each component to its sign, Section 2).
2. With a = |P_K(wbar)|^2 the remaining m-problem is
   h(m) = a/(2(m + tau)) + F(m) + (m - mbar)^2/(2 tau) + const, m >= 0,
   which is strictly convex with
   h'(m) = -a/(2(m+tau)^2) + c2 m^2 + (c1 + 1/tau) m + V - mbar/tau.
3. If h'(0) >= 0, i.e. 2 tau^2 V - 2 tau mbar - a >= 0, then m = 0 and w = 0.
4. Otherwise the root of h' is found by Newton's method:
   * c2 = 0: h' is increasing and concave on m >= 0, so Newton's method
     started at the root for a = 0, max(0, (mbar - tau V)/(1 + tau c1)), which
     lies left of the root, rises monotonically towards it. Iterate while an
     update still increases m (at most 64 updates).
   * c2 > 0: h' is increasing but neither concave nor convex. Write
     Q(m) = c2 m^2 + (c1 + 1/tau) m + V - mbar/tau. Since
     -a/(2 tau^2) <= -a/(2(m+tau)^2) <= 0, the root lies between the root of Q
     (lo) and the root of Q - a/(2 tau^2) (hi), both in closed form. Newton's
     method starts at lo and keeps the bracket: each iterate replaces lo or hi
     by the sign of h', and a Newton step that leaves the open bracket is
     replaced by its midpoint. It stops when the iterate no longer moves or
     the bracket cannot be split (at most 100 steps).

General q (prox_cells_q), with a = |P_K(wbar)| (not squared):
1'. For fixed m > 0 and fixed |w| = rho the best direction in the cone is that
   of P_K(wbar), so w = rho P_K(wbar)/a; the optimal rho satisfies
   (rho/m)^(q-1) + (rho - a)/tau = 0. With s = rho/m this reads
   phi(s) = tau s^(q-1) + m s - a = 0, increasing in s, with its root in
   (0, min(a/m, s_max)], s_max = (a/tau)^(1/(q-1)) (the root at m = 0).
2'. The m-problem has the derivative (envelope theorem)
   h'(m) = -s(m)^q/q' + f(x, m) + (m - mbar)/tau, increasing in m, with
   h''(m) = (q-1) s^q/(tau (q-1) s^(q-2) + m) + f'(x, m) + 1/tau.
3'. If h'(0) = -s_max^q/q' + V - mbar/tau >= 0 then m = 0, w = 0. If a = 0,
   w = 0 and m is the non-negative root of f(x, m) + (m - mbar)/tau.
4'. Otherwise, since -s_max^q/q' <= -s^q/q' <= 0, the root of h' lies between
   the roots of Q(m) = c2 m^2 + (c1 + 1/tau) m + V - mbar/tau (lo) and of
   Q - s_max^q/q' (hi), as for q = 2. Newton's method on h' keeps that bracket
   (midpoint when a step leaves it); each h'(m) takes s(m) from Newton's method
   on phi kept in its own bracket. Both stop when the iterate no longer moves or
   the bracket cannot be split. Then w = m s P_K(wbar)/a. (Solving in m keeps m
   accurate where m is small against a/s, where m(s) = a/s - tau s^(q-2)
   cancels.)
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

MAX_NEWTON = 64
MAX_SAFE_NEWTON = 100


@dataclasses.dataclass(frozen=True)
class Coupling:
    """The per-cell costs: f(x, m) = c2 m^2 + c1 m + V(x), the terminal cost
    g(x, m) = (m - mbar_T(x))/beta (beta = 0: g = 0) and the Hamiltonian's
    exponent q' (eq. power_hamiltonian). V is passed separately."""
    c2: float = 0.0
    c1: float = 1.0
    beta: float = 0.0
    mbar_T: Optional[np.ndarray] = None
    qprime: float = 2.0

    def __post_init__(self):
        if self.c2 < 0 or self.c1 < 0:
            raise ValueError("the coupling must be non-decreasing in m (c2, c1 >= 0)")
        if self.beta < 0:
            raise ValueError("beta must be >= 0")
        if self.beta > 0 and self.mbar_T is None:
            raise ValueError("a terminal penalty needs its target density")
        if not self.qprime > 1.0:
            raise ValueError("q' must be > 1")

    @property
    def q(self) -> float:
        """Exponent of b-hat, the conjugate of q'."""
        return self.qprime / (self.qprime - 1.0)


LINEAR = Coupling()                       # f = m + V, g = 0
PROBLEM1 = Coupling(c2=0.5, c1=0.0)       # f = (m^2 + 2 V)/2 (Section 5.1)


def problem2_coupling(mbar_T: np.ndarray, beta: float = 1e-3) -> Coupling:
    """f = 0 and g = (m - mbar_T)/beta (Section 5.2)."""
    return Coupling(c2=0.0, c1=0.0, beta=beta, mbar_T=np.asarray(mbar_T, dtype=np.float64))


def cell_coefficients(g, V: np.ndarray, cost: Coupling = LINEAR):
    """Per-cell (c1, V) over the n cells of the m block (slice t holds m^{t+1}):
    the coupling's values, with the terminal term added on the last slice."""
    c1 = np.full(g.n, float(cost.c1))
    Vt = np.tile(np.asarray(V, dtype=np.float64), g.nt)
    if cost.beta > 0:
        w = 1.0 / (cost.beta * g.dt)
        last = slice((g.nt - 1) * g.M, g.n)
        c1[last] += w
        Vt[last] = Vt[last] - w * np.asarray(cost.mbar_T, dtype=np.float64)
    return c1, Vt


def project_cone(wbar: np.ndarray) -> np.ndarray:
    """P_K applied to an array of shape (2d, ...): even components are clipped
    to [0, inf), odd ones to (-inf, 0]."""
    w = np.array(wbar, dtype=np.float64, copy=True)
    w[0::2] = np.maximum(w[0::2], 0.0)
    w[1::2] = np.minimum(w[1::2], 0.0)
    return w


def _quad_root(c2, B, C):
    """Non-negative root of c2 m^2 + B m + C (B > 0, c2 > 0), 0 when C >= 0;
    written without cancellation."""
    disc = np.sqrt(B * B - 4.0 * c2 * np.minimum(C, 0.0))
    return np.where(C < 0.0, -2.0 * C / (B + disc), 0.0)


def prox_cells(mbar: np.ndarray, wbar: np.ndarray, V: np.ndarray, tau: float,
               return_iters: bool = False, c1=1.0, c2: float = 0.0):
    """Vectorised per-cell prox. mbar, V, c1: shape (N,) (V and c1 broadcast);
    wbar: shape (2d, N); c2 a scalar. Returns (m, w) (and the Newton update
    count per cell if asked)."""
    mbar = np.asarray(mbar, dtype=np.float64)
    V = np.broadcast_to(np.asarray(V, dtype=np.float64), mbar.shape)
    c1 = np.broadcast_to(np.asarray(c1, dtype=np.float64), mbar.shape)
    wt = project_cone(wbar)
    a = np.sum(wt * wt, axis=0)
    zero = (2.0 * tau * tau * V - 2.0 * tau * mbar - a) >= 0.0
    iters = np.zeros(mbar.shape, dtype=np.int64)
    active = ~zero
    B = c1 + 1.0 / tau
    if c2 == 0.0:
        m = np.maximum(0.0, (mbar - tau * V) / (1.0 + tau * c1))
        for _ in range(MAX_NEWTON):
            if not active.any():
                break
            s = m + tau
            hp = -a / (2.0 * s * s) + B * m + V - mbar / tau
            hpp = a / (s * s * s) + B
            m_new = m - hp / hpp
            up = active & (m_new > m)
            m = np.where(up, m_new, m)
            iters += up
            active = up
    else:
        C = V - mbar / tau
        lo = _quad_root(c2, B, C)
        hi = _quad_root(c2, B, C - a / (2.0 * tau * tau))
        m = lo.copy()
        for _ in range(MAX_SAFE_NEWTON):
            if not active.any():
                break
            s = m + tau
            hp = -a / (2.0 * s * s) + (c2 * m + B) * m + C
            hpp = a / (s * s * s) + 2.0 * c2 * m + B
            lo = np.where(active & (hp < 0.0), m, lo)
            hi = np.where(active & (hp > 0.0), m, hi)
            mn = m - hp / hpp
            outside = ~((mn > lo) & (mn < hi))
            mid = 0.5 * (lo + hi)
            mn = np.where(outside, mid, mn)
            stuck = outside & ((mid <= lo) | (mid >= hi))
            move = active & (hp != 0.0) & ~stuck & (mn != m)
            m = np.where(move, mn, m)
            iters += move
            active = move
    m = np.where(zero, 0.0, m)
    w = (m / (m + tau)) * wt
    w[:, zero] = 0.0
    if return_iters:
        return m, w, iters
    return m, w


def _bracketed_newton(F, lo, hi, x, active, max_iter=200):
    """Vectorised Newton's method for an increasing function, kept in [lo, hi]:
    F(x) -> (value, derivative); a step that leaves the open bracket is replaced
    by its midpoint; each entry stops when it no longer moves or its bracket
    cannot be split."""
    for _ in range(max_iter):
        if not active.any():
            break
        val, der = F(x)
        lo = np.where(active & (val < 0.0), x, lo)
        hi = np.where(active & (val > 0.0), x, hi)
        with np.errstate(divide="ignore", invalid="ignore"):
            xn = x - val / der
        out = ~((xn > lo) & (xn < hi))
        mid = 0.5 * (lo + hi)
        xn = np.where(out, mid, xn)
        stuck = out & ((mid <= lo) | (mid >= hi))
        move = active & (val != 0.0) & ~stuck & (xn != x)
        x = np.where(move, xn, x)
        active = move
    return x


def prox_cells_q(mbar: np.ndarray, wbar: np.ndarray, V: np.ndarray, tau: float, q: float,
                 c1=1.0, c2: float = 0.0):
    """Per-cell prox for a general exponent q of b-hat (steps 1'-4'), vectorised
    over cells; shapes as in prox_cells. Returns (m, w)."""
    qp = q / (q - 1.0)
    mbar = np.asarray(mbar, dtype=np.float64)
    V = np.broadcast_to(np.asarray(V, dtype=np.float64), mbar.shape)
    c1 = np.broadcast_to(np.asarray(c1, dtype=np.float64), mbar.shape)
    wt = project_cone(wbar)
    a = np.sqrt(np.sum(wt * wt, axis=0))
    B = c1 + 1.0 / tau
    C = V - mbar / tau

    def root_Q(Cc):
        return _quad_root(c2, B, Cc) if c2 > 0 else np.maximum(0.0, -Cc / B)

    has = a > 0
    ap = np.where(has, a, 1.0)
    smax = (ap / tau) ** (1.0 / (q - 1.0))
    hmax = smax ** q / qp
    act = has & (-hmax + C < 0.0)          # h'(0) < 0
    state = {"s": smax.copy()}

    def s_of(m):
        # root of phi(s) = tau s^(q-1) + m s - a in (0, min(a/m, s_max)]
        cap = np.where(m > 0, np.minimum(ap / np.where(m > 0, m, 1.0), smax), smax)
        s0 = np.minimum(state["s"], cap)    # from the previous m (always > 0)

        def phi(s):
            return tau * s ** (q - 1.0) + m * s - ap, tau * (q - 1.0) * s ** (q - 2.0) + m

        s = _bracketed_newton(phi, np.zeros_like(cap), cap, s0, act.copy())
        state["s"] = s
        return s

    def hprime(m):
        s = s_of(m)
        sq = s ** q
        val = -sq / qp + (c2 * m + B) * m + C
        der = (q - 1.0) * sq / (tau * (q - 1.0) * s ** (q - 2.0) + m) + 2.0 * c2 * m + B
        return val, der

    lo = root_Q(C)
    hi = root_Q(C - hmax)
    m = _bracketed_newton(hprime, lo.copy(), hi.copy(), lo.copy(), act.copy())
    s = s_of(m)
    m_a0 = root_Q(C)                       # a = 0: w = 0
    m = np.where(act, m, np.where(has, 0.0, m_a0))
    w = np.where(act, m * s / ap, 0.0) * wt
    return m, w


def prox_primal(g, y: np.ndarray, V: np.ndarray, tau: float,
                cost: Coupling = LINEAR) -> np.ndarray:
    """prox_{tau phi} on a whole primal vector y = (m, w^(0..2d-1)), each block
    of N_t x M values; V (length M) is the same at every time slice."""
    nb = 1 + g.ncomp
    Y = y.reshape(nb, g.nt * g.M)
    c1, Vt = cell_coefficients(g, V, cost)
    if cost.qprime == 2.0:
        m, w = prox_cells(Y[0], Y[1:], Vt, tau, c1=c1, c2=cost.c2)
    else:
        m, w = prox_cells_q(Y[0], Y[1:], Vt, tau, cost.q, c1=c1, c2=cost.c2)
    return np.concatenate([m[None], w], axis=0).reshape(-1)


def cell_objective(m, w, mbar, wbar, V, tau, c1=1.0, c2=0.0, q=2.0):
    """Per-cell objective of the prox problem (for checks); b-hat with exponent q."""
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
        bh = float(np.dot(w, w)) ** (q / 2.0) / (q * m ** (q - 1.0))
    F = c2 * m ** 3 / 3.0 + 0.5 * c1 * m * m + V * m
    return bh + F + ((m - mbar) ** 2 + float(np.dot(w - wbar, w - wbar))) / (2.0 * tau)
