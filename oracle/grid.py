"""Discretisation parameters (Section 2).

Periodic: dx = (b - a) / N_x, nodes a + i dx for i = 0..N_x-1 (torus grid).
Neumann:  dx = (b - a) / (N_x + 1), interior nodes a + i dx for i = 1..N_x
          (the number of unknowns is the same for both boundary types).
Time:     dt = T / N_t, t_k = k dt for k = 0..N_t.

The boundary type is set per axis (Section 4.3 notes that the spatial solver
allows different conditions in x and y): bc is "periodic", "neumann" (every
axis) or, for d = 2, a pair (bc_x, bc_y). Each axis then takes the spacing,
the one-axis operators and the spatial transform of its own type.
"""
from __future__ import annotations

import dataclasses


@dataclasses.dataclass(frozen=True)
class Grid:
    d: int
    nx: int
    ny: int
    nt: int
    bc: object            # "periodic" | "neumann" | (bc_x, bc_y) when d = 2
    nu: float
    T: float = 1.0
    lo: tuple = (0.0, 0.0)
    hi: tuple = (1.0, 1.0)
    l: int = 1
    gamma: float = 5e-4

    def __post_init__(self):
        if self.d not in (1, 2):
            raise ValueError("d must be 1 or 2")
        if self.d == 1 and self.ny != 1:
            raise ValueError("d = 1 uses ny = 1")
        kinds = ("periodic", "neumann")
        if isinstance(self.bc, tuple):
            if self.d != 2 or len(self.bc) != 2 or any(b not in kinds for b in self.bc):
                raise ValueError("a per-axis bc is a pair (bc_x, bc_y) of periodic/neumann, d = 2")
        elif self.bc not in kinds:
            raise ValueError("bc must be periodic or neumann")

    @property
    def bcs(self) -> tuple:
        """Boundary type of each axis, (x, y) (y repeats x when d = 1)."""
        return self.bc if isinstance(self.bc, tuple) else (self.bc, self.bc)

    @property
    def dt(self) -> float:
        return self.T / self.nt

    @staticmethod
    def _h(N, a, b, bc):
        return (b - a) / N if bc == "periodic" else (b - a) / (N + 1)

    @property
    def dx(self) -> float:
        return self._h(self.nx, self.lo[0], self.hi[0], self.bcs[0])

    @property
    def dy(self) -> float:
        if self.d == 1:
            return 1.0
        return self._h(self.ny, self.lo[1], self.hi[1], self.bcs[1])

    @property
    def M(self) -> int:
        return self.nx * self.ny

    @property
    def n(self) -> int:
        return self.nt * self.M

    @property
    def ncomp(self) -> int:
        """Number of flux components w^(c): 2d (Section 2, [D_h] and div_h)."""
        return 2 * self.d


def grid_from(params: dict) -> Grid:
    """Build a Grid from a plain parameter dict (keys as in Grid)."""
    d = params["d"]
    lo = tuple(params.get("lo", (0.0,) * d)) + (0.0,) * (2 - d)
    hi = tuple(params.get("hi", (1.0,) * d)) + (1.0,) * (2 - d)
    bc = params["bc"]
    bc = tuple(bc) if isinstance(bc, (list, tuple)) else bc
    return Grid(d=d, nx=params["nx"], ny=params.get("ny", 1), nt=params["nt"],
                bc=bc, nu=params["nu"], T=params.get("T", 1.0),
                lo=lo, hi=hi, l=params.get("l", 1), gamma=params.get("gamma", 5e-4))
