"""Seeded synthetic inputs for the variational MFG solver.

This module only draws problem data (the potential V in the coupling
f(x, m) = m + V(x), and the initial density m0) from seeded generators. It
holds none of the solver's arithmetic, so both the plain CPU checker and the
GPU path can take their inputs from here without sharing any method code.

The paper's own workloads are analytic (Section 5.1, Problem 1; Section 5.2,
Problem 2) and are given here without random draws (paper_problem1/2). The
other shapes below follow the configurations the GPU library is
measured on: a 1-D torus with 64 nodes and 32 time steps, a 128x128 torus with
64 time steps, the 256x256 Neumann square with 128 time steps, a batch of 32
uneven periodic instances, and a 256x256 torus with 100 time steps for the
gradient. Draw order is fixed and documented per function; every array is
float64 in [i][j] order (j fastest).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

PERIODIC = "periodic"
NEUMANN = "neumann"


@dataclasses.dataclass
class Instance:
    """One problem instance: grid, parameters and the two input fields."""
    d: int
    nx: int
    ny: int            # 1 when d == 1
    nt: int
    bc: object         # "periodic" or "neumann" (both axes), or (bc_x, bc_y)
    nu: float
    gamma: float
    T: float
    lo: tuple
    hi: tuple
    V: np.ndarray      # potential, shape (nx*ny,)
    m0: np.ndarray     # initial density, shape (nx*ny,)
    l: int = 1         # time preconditioner: 1 = DCT-VIII, 2 = DST-I
    name: str = ""

    @property
    def M(self) -> int:
        return self.nx * self.ny

    @property
    def n(self) -> int:
        return self.nt * self.nx * self.ny

    def params(self) -> dict:
        """Plain parameter dict (no arrays)."""
        return dict(d=self.d, nx=self.nx, ny=self.ny, nt=self.nt, bc=self.bc,
                    nu=self.nu, gamma=self.gamma, T=self.T, lo=self.lo,
                    hi=self.hi, l=self.l)


def node_coords(N: int, bc: str, a: float = 0.0, b: float = 1.0) -> np.ndarray:
    """Grid nodes along one axis: a + i*dx, i < N (periodic, dx = (b-a)/N) or
    i = 1..N (Neumann interior nodes, dx = (b-a)/(N+1)); Section 2."""
    if bc == PERIODIC:
        return a + (b - a) * np.arange(N) / N
    return a + (b - a) * np.arange(1, N + 1) / (N + 1)


def axis_bcs(bc) -> tuple:
    """(bc_x, bc_y) of a boundary specification (one type, or a per-axis pair)."""
    return tuple(bc) if isinstance(bc, (tuple, list)) else (bc, bc)


def _mesh(d, nx, ny, bc):
    bx, by = axis_bcs(bc)
    x = node_coords(nx, bx)
    if d == 1:
        return [x]
    y = node_coords(ny, by)
    X, Y = np.meshgrid(x, y, indexing="ij")
    return [X, Y]


def gaussian_mixture(rng: np.random.Generator, d: int, nx: int, ny: int, bc: str,
                     K: int) -> np.ndarray:
    """K equal-weight Gaussian bumps; centres ~ U[0,1)^d then widths ~ U[0.05,0.15].
    Periodic distances use the minimal image. Normalised so dx^d * sum = 1."""
    centres = rng.uniform(0.0, 1.0, size=(K, d))
    sigmas = rng.uniform(0.05, 0.15, size=K)
    coords = _mesh(d, nx, ny, bc)
    bcs = axis_bcs(bc)
    out = np.zeros(coords[0].shape)
    for r in range(K):
        dist2 = np.zeros_like(out)
        for ax in range(d):
            delta = coords[ax] - centres[r, ax]
            if bcs[ax] == PERIODIC:
                delta = delta - np.round(delta)
            dist2 += delta * delta
        out += np.exp(-dist2 / (2.0 * sigmas[r] ** 2))
    dx = (1.0 / nx) if bcs[0] == PERIODIC else 1.0 / (nx + 1)
    dy = 1.0 if d == 1 else ((1.0 / ny) if bcs[1] == PERIODIC else 1.0 / (ny + 1))
    out /= out.sum() * dx * dy
    return out.reshape(-1).astype(np.float64)


def cosine_modes_neumann(rng: np.random.Generator, nx: int, ny: int, amp: float = 0.5,
                         count: int = 8) -> np.ndarray:
    """amp * sum_r a_r cos(pi p_r x) cos(pi q_r y) / max|.|; (p_r, q_r) drawn
    without replacement from {0..3}^2 minus (0,0) (lexicographic list), then
    a_r ~ U[-1, 1]. Cosine modes satisfy the no-flux condition."""
    pairs = [(p, q) for p in range(4) for q in range(4) if (p, q) != (0, 0)]
    idx = rng.choice(len(pairs), size=count, replace=False)
    a = rng.uniform(-1.0, 1.0, size=count)
    X, Y = _mesh(2, nx, ny, NEUMANN)
    field = np.zeros_like(X)
    for r, k in enumerate(idx):
        p, q = pairs[k]
        field += a[r] * np.cos(np.pi * p * X) * np.cos(np.pi * q * Y)
    field *= amp / np.abs(field).max()
    return field.reshape(-1)


def periodic_modes(rng: np.random.Generator, nx: int, ny: int, amp: float = 0.5,
                   count: int = 8) -> np.ndarray:
    """amp-normalised sum of cos(2 pi (p x + q y) + phi); (p, q) drawn without
    replacement from {-3..3}^2 minus (0,0) (lexicographic list), then
    phi ~ U[0, 2 pi)."""
    pairs = [(p, q) for p in range(-3, 4) for q in range(-3, 4) if (p, q) != (0, 0)]
    idx = rng.choice(len(pairs), size=count, replace=False)
    phi = rng.uniform(0.0, 2.0 * np.pi, size=count)
    X, Y = _mesh(2, nx, ny, PERIODIC)
    field = np.zeros_like(X)
    for r, k in enumerate(idx):
        p, q = pairs[k]
        field += np.cos(2.0 * np.pi * (p * X + q * Y) + phi[r])
    field *= amp / np.abs(field).max()
    return field.reshape(-1)


def _bounds(d):
    return (0.0,) * d, (1.0,) * d


def torus_1d(seed: int = 1, nx: int = 64, nt: int = 32, nu: float = 0.1) -> Instance:
    """1-D torus, V = 0.5 sin(2 pi x), m0 = mixture of 3 bumps (seed 1 by default)."""
    rng = np.random.default_rng(seed)
    x = node_coords(nx, PERIODIC)
    V = 0.5 * np.sin(2.0 * np.pi * x)
    m0 = gaussian_mixture(rng, 1, nx, 1, PERIODIC, 3)
    lo, hi = _bounds(1)
    return Instance(1, nx, 1, nt, PERIODIC, nu, 5e-4, 1.0, lo, hi, V, m0,
                    name=f"torus1d_{nx}x{nt}")


def torus_2d_trig(seed: int = 2, n: int = 128, nt: int = 64, nu: float = 1e-2) -> Instance:
    """2-D torus, V = sin(2 pi x) cos(2 pi y), m0 = mixture of 5 bumps."""
    rng = np.random.default_rng(seed)
    X, Y = _mesh(2, n, n, PERIODIC)
    V = (np.sin(2.0 * np.pi * X) * np.cos(2.0 * np.pi * Y)).reshape(-1)
    m0 = gaussian_mixture(rng, 2, n, n, PERIODIC, 5)
    lo, hi = _bounds(2)
    return Instance(2, n, n, nt, PERIODIC, nu, 5e-4, 1.0, lo, hi, V, m0,
                    name=f"torus2d_{n}x{n}x{nt}_nu{nu:g}")


def neumann_square(seed: int = 3, n: int = 256, nt: int = 128, nu: float = 1e-2) -> Instance:
    """Neumann unit square; V = 8 random cosine modes (amplitude 0.5), then
    m0 = mixture of 5 bumps."""
    rng = np.random.default_rng(seed)
    V = cosine_modes_neumann(rng, n, n)
    m0 = gaussian_mixture(rng, 2, n, n, NEUMANN, 5)
    lo, hi = _bounds(2)
    return Instance(2, n, n, nt, NEUMANN, nu, 5e-3, 1.0, lo, hi, V, m0,
                    name=f"neumann2d_{n}x{n}x{nt}_nu{nu:g}")


def batch_instance(i: int, base_seed: int = 4) -> Instance:
    """Instance i of the uneven periodic batch, rng = default_rng([4, i]):
    grid from {64,96,128,192,256}, N_t from {32,64,100,128}, log10 nu ~ U[-3,0],
    then V (8 periodic modes, amplitude 0.5), then m0 (5 bumps)."""
    rng = np.random.default_rng([base_seed, i])
    n = int(rng.choice([64, 96, 128, 192, 256]))
    nt = int(rng.choice([32, 64, 100, 128]))
    nu = float(10.0 ** rng.uniform(-3.0, 0.0))
    V = periodic_modes(rng, n, n)
    m0 = gaussian_mixture(rng, 2, n, n, PERIODIC, 5)
    lo, hi = _bounds(2)
    return Instance(2, n, n, nt, PERIODIC, nu, 5e-4, 1.0, lo, hi, V, m0,
                    name=f"batch{i}_{n}x{n}x{nt}")


def gradient_instance(seed: int = 5, n: int = 256, nt: int = 100, nu: float = 5e-2):
    """2-D torus for the gradient workload: V (8 periodic modes), m0 (5 bumps),
    then the target density m_target (5 bumps). Returns (Instance, m_target)."""
    rng = np.random.default_rng(seed)
    V = periodic_modes(rng, n, n)
    m0 = gaussian_mixture(rng, 2, n, n, PERIODIC, 5)
    m_target = gaussian_mixture(rng, 2, n, n, PERIODIC, 5)
    lo, hi = _bounds(2)
    inst = Instance(2, n, n, nt, PERIODIC, nu, 5e-4, 1.0, lo, hi, V, m0,
                    name=f"grad_{n}x{n}x{nt}")
    return inst, m_target


def small_instance(seed: int, d: int, nx: int, ny: int, nt: int, bc: str, nu: float,
                   l: int = 1, K: int = 3, gamma: Optional[float] = None) -> Instance:
    """Small ragged instance for parity tests: V from random modes (Neumann
    cosines or periodic modes; 1-D uses 0.5 sin(2 pi x + phi)), then m0."""
    rng = np.random.default_rng(seed)
    if d == 1:
        phi = rng.uniform(0.0, 2.0 * np.pi)
        x = node_coords(nx, bc)
        V = 0.5 * np.sin(2.0 * np.pi * x + phi)
        ny = 1
    elif bc == NEUMANN:
        V = cosine_modes_neumann(rng, nx, ny)
    else:
        V = periodic_modes(rng, nx, ny)
    m0 = gaussian_mixture(rng, d, nx, ny, bc, K)
    lo, hi = _bounds(d)
    if gamma is None:
        gamma = 5e-4 if bc == PERIODIC else 5e-3
    return Instance(d, nx, ny, nt, bc, nu, gamma, 1.0, lo, hi, V, m0, l=l,
                    name=f"small_{d}d_{bc}_{nx}x{ny}x{nt}")


def mixed_instance(seed: int, nx: int, ny: int, nt: int, bc_x: str, bc_y: str, nu: float,
                   l: int = 1, K: int = 3, gamma: float = 5e-3, amp: float = 0.5,
                   count: int = 6) -> Instance:
    """2-D instance with a boundary type per axis. V = amp-normalised sum of
    count products phi_p(x) psi_q(y), each factor cos(2 pi p x + phase) on a
    periodic axis and cos(pi p x) on a Neumann axis (so V respects both
    conditions); draws: (p, q) from {0..3}^2 minus (0,0) without replacement
    (lexicographic list), then the coefficients ~ U[-1, 1], then the phases
    ~ U[0, 2 pi) (x then y per term), then m0 (K bumps, minimal image on the
    periodic axis only)."""
    rng = np.random.default_rng(seed)
    bc = (bc_x, bc_y)
    pairs = [(p, q) for p in range(4) for q in range(4) if (p, q) != (0, 0)]
    idx = rng.choice(len(pairs), size=count, replace=False)
    a = rng.uniform(-1.0, 1.0, size=count)
    ph = rng.uniform(0.0, 2.0 * np.pi, size=(count, 2))
    X, Y = _mesh(2, nx, ny, bc)

    def factor(z, k, kind, phase):
        return np.cos(2.0 * np.pi * k * z + phase) if kind == PERIODIC else np.cos(np.pi * k * z)

    field = np.zeros_like(X)
    for r, kk in enumerate(idx):
        p, q = pairs[kk]
        field += a[r] * factor(X, p, bc_x, ph[r, 0]) * factor(Y, q, bc_y, ph[r, 1])
    V = (field * amp / np.abs(field).max()).reshape(-1)
    m0 = gaussian_mixture(rng, 2, nx, ny, bc, K)
    lo, hi = _bounds(2)
    return Instance(2, nx, ny, nt, bc, nu, gamma, 1.0, lo, hi, V, m0, l=l,
                    name=f"mixed_{bc_x[0]}{bc_y[0]}_{nx}x{ny}x{nt}")


def paper_problem1(n: int, nt: int, nu: float) -> Instance:
    """Problem 1 of Section 5.1 on the unit torus (d = 2, N_x = N_y = n): the
    coupling f = (m^2 - sin 2 pi y - sin 2 pi x - cos 4 pi x)/2, written as
    m^2/2 + V with V = -(sin 2 pi y + sin 2 pi x + cos 4 pi x)/2; m0 = 1; g = 0;
    gamma = 5e-4. x is axis 0 (i), y axis 1 (j). No random draws."""
    X, Y = _mesh(2, n, n, PERIODIC)
    V = -0.5 * (np.sin(2.0 * np.pi * Y) + np.sin(2.0 * np.pi * X) + np.cos(4.0 * np.pi * X))
    m0 = np.ones(n * n)
    lo, hi = _bounds(2)
    return Instance(2, n, n, nt, PERIODIC, nu, 5e-4, 1.0, lo, hi, V.reshape(-1), m0,
                    name=f"problem1_{n}x{n}x{nt}_nu{nu:g}")


def paper_problem2(n: int, nt: int, nu: float):
    """Problem 2 of Section 5.2: Neumann on [-1/2, 1/2]^2 (interior nodes
    -1/2 + i/(n+1), i = 1..n), f = 0 (V = 0), gamma = 5e-3, and the Gaussians
    m0 = 3 exp(-2^7 ((x + 1/4)^2 + (y - 1/4)^2)) and the target
    mbar = 3 exp(-2^7 ((x - 1/4)^2 + (y + 1/4)^2)) of the terminal penalty
    g = (m - mbar)/beta, beta = 1e-3. No random draws.
    Returns (Instance, mbar, beta)."""
    x = node_coords(n, NEUMANN, -0.5, 0.5)
    X, Y = np.meshgrid(x, x, indexing="ij")
    m0 = 3.0 * np.exp(-128.0 * ((X + 0.25) ** 2 + (Y - 0.25) ** 2))
    mbar = 3.0 * np.exp(-128.0 * ((X - 0.25) ** 2 + (Y + 0.25) ** 2))
    inst = Instance(2, n, n, nt, NEUMANN, nu, 5e-3, 1.0, (-0.5, -0.5), (0.5, 0.5),
                    np.zeros(n * n), m0.reshape(-1), name=f"problem2_{n}x{n}x{nt}_nu{nu:g}")
    return inst, mbar.reshape(-1), 1e-3


def random_vector(seed: int, size: int) -> np.ndarray:
    """Seeded N(0,1) vector (right-hand sides, operator inputs)."""
    return np.random.default_rng(seed).standard_normal(size)
