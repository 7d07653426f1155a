"""Discretisation parameters (Section 2).

Periodic: dx = (b - a) / N_x, nodes a + i dx for i = 0..N_x-1 (torus grid).
Neumann:  dx = (b - a) / (N_x + 1), interior nodes a + i dx for i = 1..N_x
          (the number of unknowns is the same for both boundary types).
Time:     dt = T / N_t, t_k = k dt for k = 0..N_t.
"""
from __future__ import annotations

import dataclasses


@dataclasses.dataclass(frozen=True)
class Grid:
    d: int
    nx: int
    ny: int
    nt: int
    bc: str               # "periodic" | "neumann"
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
        if self.bc not in ("periodic", "neumann"):
            raise ValueError("bc must be periodic or neumann")

    @property
    def dt(self) -> float:
        return self.T / self.nt

    def _h(self, N, a, b):
        return (b - a) / N if self.bc == "periodic" else (b - a) / (N + 1)

    @property
    def dx(self) -> float:
        return self._h(self.nx, self.lo[0], self.hi[0])

    @property
    def dy(self) -> float:
        if self.d == 1:
            return 1.0
        return self._h(self.ny, self.lo[1], self.hi[1])

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
    return Grid(d=d, nx=params["nx"], ny=params.get("ny", 1), nt=params["nt"],
                bc=params["bc"], nu=params["nu"], T=params.get("T", 1.0),
                lo=lo, hi=hi, l=params.get("l", 1), gamma=params.get("gamma", 5e-4))
