"""Seeded, synthetic problem descriptions for the time-periodic eddy-current problem.

This module is the only code shared by the CPU oracle and the GPU path. It holds
problem *descriptions* (geometry rectangles, material-law parameters, source
amplitude, grid and time sizes) and seeded random draws. It contains none of the
method's arithmetic: no mesh, no assembly, no operator, no solver.

The problem (Sec. 4 of the paper, "Test problem"): find the z-component u of the
magnetic vector potential on the unit square with u = 0 on the boundary and

    sigma * du/dt - div(nu(|grad u|) grad u) = j,   T-periodic in time,

discretised by P1 finite elements on a uniform grid (each square split along the
SW-NE diagonal) and by implicit Euler with N steps per period (Problem 1,
eqs. (disc1)-(disc2)). The synthetic stand-in for the paper's transformer
cross-section keeps its structure: a nonlinear iron region, a current-driven coil
strip and a conducting block where sigma > 0 (sigma = 0 elsewhere, so the mass
operator is degenerate, assumption (A2)).

Material law inside the iron rectangle:  nu(s) = theta * (nu_a + nu_b s^2/(1+s^2)),
outside:                                   nu(s) = theta * nu_out,
where theta is an optional per-triangle scale (1 by default).
Source: f(x, t) = J0 * w(2 pi t / T) on the coil rectangle, w = sin (or cos).
Linear part of the fixed-point iteration: Khat = nu_max * (P1 stiffness).
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field, replace
from typing import List, Optional, Tuple

import numpy as np

__all__ = [
    "Rect", "Problem", "config1", "config2", "config3", "config4", "config5",
    "with_size", "random_field", "manufactured_coeffs", "CONFIG1_TOL",
]


@dataclass(frozen=True)
class Rect:
    """Closed axis-aligned rectangle [x0, x1] x [y0, y1]."""
    x0: float
    y0: float
    x1: float
    y1: float

    def as_tuple(self) -> Tuple[float, float, float, float]:
        return (self.x0, self.y0, self.x1, self.y1)


@dataclass(frozen=True)
class Problem:
    """Description of one time-periodic problem instance.

    Grid: n x n square cells of side h = 1/n on the unit square, (n+1)^2 nodes.
    Time: N implicit-Euler steps per period T, tau = T/N, t_n = n tau, n = 1..N.
    """
    n: int = 32
    N: int = 32
    T: float = 1.0
    sigma_in: float = 1.0
    sigma_rect: Rect = Rect(0.25, 0.25, 0.75, 0.75)
    nu_a: float = 1.0
    nu_b: float = 9.0
    nu_out: float = 1.0
    nu_rect: Rect = Rect(0.3, 0.05, 0.7, 0.95)
    J0: float = 10.0
    coil_rect: Rect = Rect(0.1, 0.3, 0.2, 0.7)
    waveform: str = "sin"        # "sin" or "cos"
    nu_max: float = 10.0
    # Optional per-triangle nu scale theta (length 2 n^2, ordering tri = 2 (j n + i) + {0, 1}).
    theta: Optional[np.ndarray] = field(default=None, compare=False, repr=False)

    @property
    def tau(self) -> float:
        return self.T / self.N

    @property
    def nodes(self) -> int:
        return (self.n + 1) ** 2

    @property
    def free_nodes(self) -> int:
        return (self.n - 1) ** 2

    @property
    def st_dofs(self) -> int:
        """Space-time degrees of freedom: free nodes times time slices."""
        return self.free_nodes * self.N


CONFIG1_TOL = 1e-10


def config1() -> Problem:
    """Plain method, FP64, small: 32 x 32 cells, N = 32, J0 = 10, unjittered iron block."""
    return Problem(n=32, N=32)


def _seeded_materials(seed: int) -> Tuple[float, Rect]:
    """Draw order: J0 = 10**U(0, 2), then a U(-0.05, 0.05) jitter of the four iron
    rectangle coordinates (x0, y0, x1, y1)."""
    rng = np.random.default_rng(seed)
    J0 = float(10.0 ** rng.uniform(0.0, 2.0))
    jit = rng.uniform(-0.05, 0.05, 4)
    base = Rect(0.3, 0.05, 0.7, 0.95)
    iron = Rect(base.x0 + jit[0], base.y0 + jit[1], base.x1 + jit[2], base.y1 + jit[3])
    return J0, iron


def config2(seed: int = 0) -> Problem:
    """256 x 256 cells (66,049 nodes), N = 256, seeded J0 and iron jitter."""
    J0, iron = _seeded_materials(seed)
    return Problem(n=256, N=256, J0=J0, nu_rect=iron)


def config3(seed: Optional[int] = 0) -> Problem:
    """1024 x 1024 cells (1,050,625 nodes), N = 512. seed=None gives the unjittered J0 = 10 case."""
    if seed is None:
        return Problem(n=1024, N=512)
    J0, iron = _seeded_materials(seed)
    return Problem(n=1024, N=512, J0=J0, nu_rect=iron)


def config4(seed: int = 0, count: int = 64) -> List[Problem]:
    """Batch of independent instances: n from {64,128,256,512}, N from {64,128,256},
    J0 log-uniform in [1, 100], iron rectangle with random corners inside [0.2, 0.8]^2."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.choice([64, 128, 256, 512]))
        N = int(rng.choice([64, 128, 256]))
        J0 = float(10.0 ** rng.uniform(0.0, 2.0))
        xs = np.sort(rng.uniform(0.2, 0.8, 2))
        ys = np.sort(rng.uniform(0.2, 0.8, 2))
        out.append(Problem(n=n, N=N, J0=J0, nu_rect=Rect(xs[0], ys[0], xs[1], ys[1])))
    return out


def config5(seed: int = 0, n: int = 256, N: int = 256) -> Problem:
    """Differentiation-mode instance: per-triangle log-normal nu scale with sd 0.1
    (constant on each square cell, so one value per cell, repeated for its two triangles)."""
    rng = np.random.default_rng(seed)
    cell = np.exp(rng.normal(0.0, 0.1, n * n))
    theta = np.repeat(cell, 2)
    return Problem(n=n, N=N, theta=theta)


def with_size(p: Problem, n: int, N: int) -> Problem:
    """Same materials and source on another grid / number of time steps."""
    theta = None
    if p.theta is not None:
        if p.n != n:
            raise ValueError("cannot resize a problem with a per-triangle theta field")
        theta = p.theta
    return replace(p, n=n, N=N, theta=theta)


def random_field(N: int, n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """Seeded random space-time field U[N, n+1, n+1] (float64) with zero boundary ring."""
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((N, n + 1, n + 1)) * scale
    U[:, 0, :] = 0.0
    U[:, -1, :] = 0.0
    U[:, :, 0] = 0.0
    U[:, :, -1] = 0.0
    return U


def manufactured_coeffs(seed: int = 0) -> Tuple[float, float, float]:
    """Coefficients (a, b, c) of a manufactured discrete solution
    u*(x, y, t) = sin(pi x) sin(pi y) (a + b cos(2 pi t / T) + c sin(4 pi t / T))."""
    rng = np.random.default_rng(seed)
    a, b, c = rng.uniform(0.05, 0.5, 3)
    return float(a), float(b), float(c)
